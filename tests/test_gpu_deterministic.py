"""Deterministic parents (BFS_DETERMINISTIC): every reached vertex other than the
root gets the least in-neighbour one level up. Parents are compared bit for bit
with the oracle's least parents computed from the oracle's levels, on symmetric
graphs (row scan, with and without sorted rows) and on directed graphs (offers
with atomicMin), alone and combined with direction-optimising runs, host
outputs and other tunables."""
import numpy as np
import pytest

import graphgen
import oracle
import paper_1604_02844_amd as bfs
from tests.gpu_helpers import gpu_run, load

pytestmark = pytest.mark.gpu

D = bfs.BFS_DETERMINISTIC
H = bfs.BFS_HYBRID


def check_least(g, dg, root, flags=D):
    print(f"[case] least parents {g.name} n={g.n} nnz={g.nnz} root={root} flags={flags}", flush=True)
    lv, pa, st = gpu_run(dg, int(root), flags)
    ref, _, _ = oracle.bfs(g.offsets, g.cols, int(root))
    assert np.array_equal(lv, ref), f"{g.name} root {root}: levels differ"
    exp = oracle.min_parents(g.offsets, g.cols, int(root), ref)
    bad = np.nonzero(pa != exp)[0]
    assert bad.size == 0, (f"{g.name} root {root}: parent of {bad[:5].tolist()} is {pa[bad[:5]].tolist()}, "
                           f"least is {exp[bad[:5]].tolist()}")
    return pa


@pytest.mark.parametrize("symmetric", [True, False])
def test_closed_forms(symmetric):
    for g, r in ((graphgen.cycle(1000), 17), (graphgen.grid(37, 53), 20 * 53 + 9), (graphgen.complete(60), 11),
                 (graphgen.star(500), 7), (graphgen.binary_tree(4095), 0), (graphgen.path(1), 0)):
        check_least(g, load(g, symmetric=symmetric), r)


@pytest.mark.parametrize("scale", [10, 14, 18])
def test_rmat_symmetric(scale):
    g = graphgen.rmat(scale, 16, seed=51 + scale)
    dg = load(g, symmetric=True)
    for r in graphgen.pick_roots(g, 4, seed=52):
        check_least(g, dg, r)
        check_least(g, dg, r, flags=D | H)


def test_rmat_loaded_without_symmetric_flag():
    """The same symmetric graph through the directed path (atomicMin offers)."""
    g = graphgen.rmat(14, 16, seed=53)
    dg = load(g, symmetric=False)
    for r in graphgen.pick_roots(g, 3, seed=54):
        check_least(g, dg, r)


def test_unsorted_rows():
    """Symmetric with rows out of order: the row scan cannot stop at the first hit."""
    rng = np.random.default_rng(55)
    n, m = 3000, 12000
    src, dst = rng.integers(0, n, m), rng.integers(0, n, m)
    g = graphgen.from_edges(n, src.tolist(), dst.tolist(), symmetric=True, dedupe=False, drop_self_loops=False,
                            sort_rows=False)
    dg = load(g, symmetric=True)
    for r in (0, 1, 2):
        check_least(g, dg, r)


def test_directed_digraphs():
    rng = np.random.default_rng(56)
    for _ in range(6):
        n = int(rng.integers(2, 5000))
        m = int(rng.integers(0, 8 * n))
        g = graphgen.from_edges(n, rng.integers(0, n, m).tolist(), rng.integers(0, n, m).tolist(),
                                symmetric=False, dedupe=False, drop_self_loops=False, sort_rows=False)
        dg = load(g)
        check_least(g, dg, int(rng.integers(0, n)))


@pytest.mark.parametrize("tun", [dict(update_mode=2), dict(block_size=256, lds_visited=-1),
                                 dict(hot_vertices=8192, block_size=1024), dict(small_max_degree=1, wave_max_degree=1)])
def test_same_parents_whatever_the_tunables(tun):
    g = graphgen.rmat(16, 16, seed=57)
    dg = load(g, symmetric=True)
    roots = graphgen.pick_roots(g, 2, seed=58)
    first = [check_least(g, dg, r) for r in roots]
    bfs.bfs_graph_set_tunables(dg, **tun)
    again = [check_least(g, dg, r, flags=D | H) for r in roots]
    for a, b in zip(first, again):
        assert np.array_equal(a, b)


def test_host_outputs_and_rmat20():
    g = graphgen.cached("rmat", scale=20, edgefactor=16, seed=1)
    dg = load(g, symmetric=True)
    r = int(graphgen.pick_roots(g, 1, seed=2)[0])
    lv = np.empty(g.n, dtype=np.int32)
    pa = np.empty(g.n, dtype=np.int32)
    bfs.bfs_run(dg, r, lv, pa, flags=D)
    ref, _, _ = oracle.bfs(g.offsets, g.cols, r)
    assert np.array_equal(lv, ref)
    assert np.array_equal(pa, oracle.min_parents(g.offsets, g.cols, r, ref))
