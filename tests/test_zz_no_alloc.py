"""GPU parity of bfs_run_noalloc (scratch in the library's static device array)
against bfs_run on the same graph and root, through the C ABI: levels
identical (and equal to the oracle's), parents valid for both (V1-V4). Two
calls in a row, the second on a smaller graph, so the second run starts from
the array the first one left; then a depth change and the degree-ordered copy;
then a run too large for the array, which is refused before any launch."""
import numpy as np
import pytest

import graphgen
import oracle
import paper_1604_02844_amd as bfs
from tests.gpu_helpers import gpu_run, load, torch_mod

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = torch_mod()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    bfs.load_library()


def noalloc_run(dg, root: int, flags: int = 0):
    torch = torch_mod()
    # Poisoned outputs: every element must be written by the run.
    lv = torch.full((dg.n,), 12345, dtype=torch.int32, device="cuda")
    pa = torch.full((dg.n,), 12345, dtype=torch.int32, device="cuda")
    bfs.bfs_run_noalloc(dg, int(root), lv, pa, flags=flags)
    return lv.cpu().numpy(), pa.cpu().numpy()


def check_against_bfs_run(g, dg, root: int, flags: int = 0):
    print(f"[case] bfs_run_noalloc {g.name} n={g.n} nnz={g.nnz} root={root} flags={flags}", flush=True)
    lv, pa = noalloc_run(dg, root, flags)
    lv_ref, pa_ref, _ = gpu_run(dg, root, flags)
    ref, _, _ = oracle.bfs(g.offsets, g.cols, int(root))
    assert np.array_equal(lv, lv_ref), f"{g.name} root {root}: levels differ from bfs_run"
    for name, (l, p) in (("noalloc", (lv, pa)), ("bfs_run", (lv_ref, pa_ref))):
        code, bad = oracle.validate(g.offsets, g.cols, int(root), ref, l, p)
        assert code == 0, f"{name} {g.name} root {root}: {oracle.CHECK_NAMES[code]} at vertex {bad}"


def test_two_calls_second_smaller():
    big = graphgen.rmat(16, 16, seed=71)
    small = graphgen.rmat(11, 16, seed=72)
    dbig, dsmall = load(big), load(small)
    rb = int(graphgen.pick_roots(big, 1, seed=73)[0])
    rs = int(graphgen.pick_roots(small, 1, seed=74)[0])
    check_against_bfs_run(big, dbig, rb)
    check_against_bfs_run(small, dsmall, rs)
    bfs.bfs_graph_free(dbig)
    bfs.bfs_graph_free(dsmall)


def test_depth_change_copy_and_hybrid():
    """A deep run after shallow ones (the first chunk of levels is sized from
    the previous call), on a graph with the degree-ordered copy (run records in
    the array), top-down and direction-optimising."""
    g = graphgen.disjoint(graphgen.rmat(13, 16, seed=75), graphgen.path(200))
    dg = load(g, symmetric=True)
    bfs.bfs_graph_set_tunables(dg, hot_vertices=512, block_size=1024)
    shallow = int(graphgen.pick_roots(graphgen.rmat(13, 16, seed=75), 1, seed=76)[0])
    for flags in (0, bfs.BFS_HYBRID):
        for r in (shallow, g.n - 1, shallow):
            check_against_bfs_run(g, dg, r, flags)
    bfs.bfs_graph_free(dg)


def test_oversized_run_refused_then_next_call_works():
    """8n bytes of run records alone exceed the array once n > 2^23: refused
    with BFS_E_NO_MEMORY, nothing written; a later call runs normally."""
    n = (bfs.BFS_NOALLOC_SCRATCH_BYTES // 8) + 4096
    g = graphgen.from_edges(n, [0, 1, 2], [1, 2, 3])
    dg = load(g)
    bfs.bfs_graph_set_tunables(dg, hot_vertices=64, block_size=1024)
    torch = torch_mod()
    lv = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    pa = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run_noalloc(dg, 0, lv, pa)
    assert e.value.status == bfs.BFS_E_NO_MEMORY
    assert int((lv != 7).sum()) == 0 and int((pa != 7).sum()) == 0
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run_noalloc(dg, n, lv, pa)
    assert e.value.status == bfs.BFS_E_ROOT_RANGE
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run_noalloc(dg, 0, lv, pa, flags=bfs.BFS_OUT_HOST)
    assert e.value.status == bfs.BFS_E_INVALID_ARG
    bfs.bfs_graph_free(dg)
    small = graphgen.rmat(10, 16, seed=77)
    check_against_bfs_run(small, load(small), int(graphgen.pick_roots(small, 1, seed=78)[0]))
