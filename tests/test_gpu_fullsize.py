"""Parity at the full workload sizes, in the launch configuration the benchmark
times: R-MAT scale 24 (every one of the 64 benchmarked roots: two against the
oracle, the rest by the V2-V5 certificate, which holds exactly when the levels
are the hop distances and the parents a BFS tree) and scale 26 (one oracle root,
eight certified), the batched configurations (R-MAT scale 22 with 64 roots,
Erdos-Renyi 2^22 with average degree 16 in batches of 8/32/64)."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import graphgen
import oracle
import paper_1604_02844_amd as bfs
from tests.gpu_helpers import check_root, gpu_run, load, torch_mod

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def certify_row(g, root, lv, pa):
    code, bad = oracle.certify(g.offsets, g.cols, int(root), lv, pa)
    assert code == 0, f"{g.name} root {root}: {oracle.CHECK_NAMES[code]} at {bad}"


def certify_runs(g, dg, roots, flags: int = 0, workers: int = 0):
    """GPU runs from every root, each certified on a host thread while the next
    runs (ctypes releases the GIL); at most `workers` outputs wait at a time."""
    workers = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    pending = []
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for r in roots:
            print(f"[case] certify {g.name} root {r} flags {flags}", flush=True)
            lv, pa, st = gpu_run(dg, int(r), flags=flags)
            assert st["reached"] == int((lv >= 0).sum())
            pending.append(ex.submit(certify_row, g, r, lv, pa))
            if len(pending) >= workers:
                pending.pop(0).result()
        for f in pending:
            f.result()


@pytest.mark.parametrize("scale,oracle_roots,cert_roots", [(24, 2, 62), (26, 1, 8)])
def test_single_root_full_scale(scale, oracle_roots, cert_roots):
    torch_mod()
    print(f"[case] generating R-MAT scale {scale}", flush=True)
    g = graphgen.cached("rmat", scale=scale, edgefactor=16, seed=1)
    dg = load(g)
    roots = graphgen.pick_roots(g, 64, seed=2)
    for r in roots[:oracle_roots]:
        check_root(g, dg, int(r))
    certify_runs(g, dg, roots[oracle_roots:oracle_roots + cert_roots], workers=8 if scale >= 26 else 0)


def test_destination_blocks_rmat24():
    """The destination-blocked expansion of the rows above T2 (off by default:
    slower at this size) at full size: 16 blocks of 2^20 vertices, one oracle
    root and seven certified, top-down."""
    torch_mod()
    g = graphgen.cached("rmat", scale=24, edgefactor=16, seed=1)
    dg = load(g)
    bfs.bfs_graph_set_tunables(dg, block_vertices=1 << 20)
    roots = graphgen.pick_roots(g, 64, seed=2)
    check_root(g, dg, int(roots[0]))
    certify_runs(g, dg, roots[1:8])


def test_hybrid_rmat24():
    """Direction-optimising runs at full size, in the configuration the hybrid
    bench times (degree-ordered copy on by default at this size)."""
    torch_mod()
    g = graphgen.cached("rmat", scale=24, edgefactor=16, seed=1)
    dg = load(g, symmetric=True)
    roots = graphgen.pick_roots(g, 64, seed=2)
    check_root(g, dg, int(roots[0]), flags=bfs.BFS_HYBRID)
    for r in roots[1:4]:
        print(f"[case] certify hybrid scale 24 root {r}", flush=True)
        lv, pa, st = gpu_run(dg, int(r), flags=bfs.BFS_HYBRID)
        certify_row(g, r, lv, pa)
        assert st["reached"] == int((lv >= 0).sum())


def test_least_parents_rmat24():
    """Deterministic parents at full size, top-down and direction-optimising."""
    torch_mod()
    g = graphgen.cached("rmat", scale=24, edgefactor=16, seed=1)
    dg = load(g, symmetric=True)
    r = int(graphgen.pick_roots(g, 64, seed=2)[0])
    ref, _, _ = oracle.bfs(g.offsets, g.cols, r)
    exp = oracle.min_parents(g.offsets, g.cols, r, ref)
    for flags in (bfs.BFS_DETERMINISTIC, bfs.BFS_DETERMINISTIC | bfs.BFS_HYBRID):
        print(f"[case] least parents scale 24 root {r} flags {flags}", flush=True)
        lv, pa, _ = gpu_run(dg, r, flags=flags)
        assert np.array_equal(lv, ref)
        assert np.array_equal(pa, exp)


def test_batch_rmat22_64_roots():
    torch = torch_mod()
    g = graphgen.cached("rmat", scale=22, edgefactor=16, seed=1)
    dg = load(g)
    roots = graphgen.pick_roots(g, 64, seed=2)
    lv = torch.empty((64, g.n), dtype=torch.int32, device="cuda")
    pa = torch.empty((64, g.n), dtype=torch.int32, device="cuda")
    print("[case] bfs_run_batch R-MAT 22, 64 roots", flush=True)
    st = bfs.bfs_run_batch(dg, roots, lv, pa)
    L, P = lv.cpu().numpy(), pa.cpu().numpy()
    for i in (0, 31, 63):
        ref, _, _ = oracle.bfs(g.offsets, g.cols, int(roots[i]))
        assert oracle.validate(g.offsets, g.cols, int(roots[i]), ref, L[i], P[i])[0] == 0
    for i, r in enumerate(roots):
        certify_row(g, r, L[i], P[i])
    assert st["reached"] == int((L >= 0).sum())


def test_batch_er22_widths():
    torch = torch_mod()
    g = graphgen.cached("er", n=1 << 22, avg_degree=16, seed=1)
    dg = load(g)
    pool = graphgen.pick_roots(g, 64, seed=2)
    for b in (8, 32, 64):
        lv = torch.empty((b, g.n), dtype=torch.int32, device="cuda")
        pa = torch.empty((b, g.n), dtype=torch.int32, device="cuda")
        print(f"[case] bfs_run_batch ER 2^22 d16, {b} roots", flush=True)
        bfs.bfs_run_batch(dg, pool[:b], lv, pa)
        L, P = lv.cpu().numpy(), pa.cpu().numpy()
        ref, _, _ = oracle.bfs(g.offsets, g.cols, int(pool[0]))
        assert oracle.validate(g.offsets, g.cols, int(pool[0]), ref, L[0], P[0])[0] == 0
        for i in range(0, b, max(1, b // 8)):
            certify_row(g, pool[i], L[i], P[i])
