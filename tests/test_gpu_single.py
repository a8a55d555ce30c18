"""GPU parity of single-root BFS (bfs_run through the C ABI) against the oracle:
levels identical, parents valid (V1-V4), run statistics equal to the oracle's."""
import numpy as np
import pytest

import graphgen
import oracle
import paper_1604_02844_amd as bfs
from tests import pins
from tests.gpu_helpers import check_root, gpu_run, load, torch_mod

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = torch_mod()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    bfs.load_library()


def test_closed_forms():
    for g, r, exp_lv, exp_par in pins.closed_form_cases():
        dg = load(g)
        lv, pa, _ = check_root(g, dg, r, expected_levels=exp_lv)
        if exp_par is not None:  # parent unique: must match exactly
            assert np.array_equal(pa, exp_par), g.name


def test_paper_examples():
    ex = pins.load_golden("paper_examples.json")
    race = ex["benign_race"]
    g = graphgen.from_edges(race["n"], *zip(*race["edges"]))
    lv, pa, _ = check_root(g, load(g), race["root"])
    assert pa[race["vertex"]] in race["valid_parents"]
    word = ex["bit_race_word"]
    g = graphgen.from_edges(word["n"], [word["root"]] * len(word["children"]), word["children"])
    lv, pa, _ = check_root(g, load(g), word["root"])
    assert all(lv[c] == 1 and pa[c] == word["root"] for c in word["children"])


def test_bitmap_layout_word_boundaries():
    """Vertices on both sides of 32-bit word boundaries (section 3.3.1 layout)."""
    n = 64 * 33 + 5
    v = np.arange(n - 1)
    g = graphgen.path(n)
    for r in (0, 31, 32, 63, 64, n - 1):
        check_root(g, load(g), r, expected_levels=np.abs(np.arange(n) - r))


def test_degenerate_graphs():
    g = graphgen.empty(1)
    lv, pa, st = gpu_run(load(g), 0)
    assert lv.tolist() == [0] and pa.tolist() == [0] and st["num_levels"] == 1
    g = graphgen.empty(100)
    lv, pa, st = gpu_run(load(g), 57)
    assert lv[57] == 0 and (lv >= 0).sum() == 1 and pa[57] == 57
    g = graphgen.disjoint(graphgen.star(40), graphgen.empty(3))
    check_root(g, load(g), 41)  # isolated root
    check_root(g, load(g), 5)


def test_self_loops_duplicates_unsorted_rows():
    rng = np.random.default_rng(5)
    n = 3000
    src = rng.integers(0, n, 20000)
    dst = rng.integers(0, n, 20000)
    g = graphgen.from_edges(n, np.r_[src, src[:500], np.arange(0, n, 7)], np.r_[dst, dst[:500], np.arange(0, n, 7)],
                            symmetric=False, dedupe=False, drop_self_loops=False, sort_rows=False)
    dg = load(g)
    for r in (0, 1, 1234):
        check_root(g, dg, r, rows_sorted=False)


@pytest.mark.parametrize("offsets_i32", [True, False])
def test_rmat_scale10_int32_csr(offsets_i32):
    """Kronecker scale 10, edgefactor 16, 16 seeded roots (the small R-MAT workload)."""
    g = graphgen.rmat(10, 16, seed=1)
    dg = load(g, offsets_i32=offsets_i32)
    for r in graphgen.pick_roots(g, 16, seed=2):
        check_root(g, dg, int(r))


def test_device_pointer_graph():
    g = graphgen.rmat(12, 16, seed=3)
    dg = load(g, device_ptrs=True)
    for r in graphgen.pick_roots(g, 4, seed=4):
        check_root(g, dg, int(r))


@pytest.mark.parametrize("tun", [
    dict(small_max_degree=1, wave_max_degree=1),                # everything grid-split or per-wavefront
    dict(small_max_degree=64, wave_max_degree=64),              # packed + grid-split rows
    dict(small_max_degree=4, wave_max_degree=100000),           # packed + wavefront, no grid split
    dict(small_max_degree=8, wave_max_degree=32),
    dict(small_max_degree=16, wave_max_degree=256, update_mode=2),   # atomicOr claims
    dict(small_max_degree=1, wave_max_degree=1, update_mode=2),
    dict(block_size=512, blocks_per_cu=1),
    dict(block_size=256, blocks_per_cu=2, update_mode=2),
    dict(block_size=512, blocks_per_cu=1, update_mode=1),
    dict(block_size=1024, blocks_per_cu=1),
    dict(hot_vertices=512),                                     # LDS hot bitmap, one hot vertex per visited word
    dict(hot_vertices=2048),                                    # capped at 1024: two per word (bits 0 and 16)
    dict(hot_vertices=2048, update_mode=2),
    dict(hot_vertices=65536, block_size=1024, small_max_degree=256),
    dict(lds_visited=1, block_size=1024),                       # whole visited bitmap in LDS
    dict(lds_visited=1, block_size=256, small_max_degree=8, wave_max_degree=32),
    dict(lds_visited=1, block_size=512, update_mode=2),
    dict(lds_visited=-1, block_size=1024),
    dict(sparse_frontier=-1),                                   # every level through the grid kernels
    dict(sparse_frontier=1),                                    # the single-workgroup path for 1-vertex frontiers only
    dict(sparse_frontier=64, update_mode=2),
    dict(hot_vertices=2048, block_vertices=2048),               # big rows grouped into 8 destination blocks
    dict(hot_vertices=2048, block_vertices=2048, update_mode=2),
    dict(hot_vertices=1024, block_vertices=4096, small_max_degree=16, wave_max_degree=64),
    dict(hot_vertices=512, block_vertices=-1),                  # copy without destination blocks
])
def test_bins_and_launch_shapes(tun):
    """Correctness does not depend on the degree bins or the launch shape."""
    g = graphgen.rmat(14, 16, seed=7)
    dg = load(g)
    bfs.bfs_graph_set_tunables(dg, **tun)
    for r in graphgen.pick_roots(g, 3, seed=8):
        check_root(g, dg, int(r))


@pytest.mark.parametrize("scale,blk,flags", [
    (16, 2048, 0),                  # 32 destination blocks
    (16, 2048, bfs.BFS_HYBRID),
    (17, 2048, 0),                  # 64 blocks, the most a row may span
    (18, 2048, 0),                  # 128 blocks: no grouping, the general path
    (17, 1 << 20, 0),               # one block holding every vertex
])
def test_destination_blocks(scale, blk, flags):
    """Rows above T2 on the degree-ordered copy grouped by destination block and
    expanded block by block (each workgroup holding one block's visited bits in
    LDS) at the large levels: levels exact, parents valid, statistics equal to
    the oracle's, top-down and direction-optimising."""
    g = graphgen.rmat(scale, 16, seed=79)
    dg = load(g, symmetric=True)
    bfs.bfs_graph_set_tunables(dg, hot_vertices=4096, block_vertices=blk, block_size=1024, wave_max_degree=128)
    assert bfs.bfs_graph_get_tunables(dg)["block_vertices"] == blk
    for r in graphgen.pick_roots(g, 4, seed=80):
        check_root(g, dg, int(r), flags=flags)
    bfs.bfs_graph_free(dg)


@pytest.mark.parametrize("scale,tun,flags", [
    (16, dict(), 0),                                      # caller's order, separate level and parent arrays
    (17, dict(update_mode=2), 0),                         # atomicOr claims beside the bins
    (17, dict(hot_vertices=2048, block_size=1024), 0),    # degree-ordered copy: one record per vertex
    (17, dict(hot_vertices=2048, block_size=1024), bfs.BFS_HYBRID),
    (18, dict(blocks_per_cu=2, block_size=256), 0),       # more expansion workgroups, smaller bin regions
    (16, dict(small_max_degree=8, wave_max_degree=16), 0),  # many rows above T2
])
def test_hub_level_bins(scale, tun, flags):
    """Hub levels (small frontier, many arcs of rows above T2) put their heads in
    destination bins that the restoration pass claims exactly in LDS: levels
    exact, parents valid, statistics equal to the oracle's, against the same
    graph with the bins off."""
    g = graphgen.rmat(scale, 16, seed=81)
    dg = load(g, symmetric=True)
    roots = [int(r) for r in graphgen.pick_roots(g, 4, seed=82)]
    deg = np.diff(g.offsets)
    roots.append(int(np.argmax(deg)))  # the largest hub as the root: binned at level 1
    for bins in (1, -1):
        # Bins are used only with the small-level path off.
        bfs.bfs_graph_set_tunables(dg, hub_bins=bins, sparse_frontier=-1, **tun)
        assert bfs.bfs_graph_get_tunables(dg)["hub_bins"] == bins
        for r in roots:
            check_root(g, dg, r, flags=flags)
    bfs.bfs_graph_free(dg)


def test_erdos_renyi():
    g = graphgen.er(1 << 16, 8, seed=9)
    dg = load(g)
    for r in graphgen.pick_roots(g, 4, seed=10):
        check_root(g, dg, int(r))


def test_contention_stress():
    """Many claimants for the same words: complete graph, star, dense id blocks."""
    for g in (graphgen.complete(300), graphgen.star(5000), graphgen.grid(64, 64)):
        dg = load(g)
        check_root(g, dg, 0)
        check_root(g, dg, g.n - 1)
    n = 4096
    a = np.repeat(np.arange(0, 64), 64)
    b = np.tile(np.arange(64, 128), 64)
    g = graphgen.from_edges(n, a, b)
    check_root(g, load(g), 0)


@pytest.mark.parametrize("update_mode", [1, 2])
def test_update_modes_scale16(update_mode):
    """Both bitmap update schemes (restoration and atomicOr) give exact levels."""
    g = graphgen.rmat(16, 16, seed=21)
    dg = load(g)
    bfs.bfs_graph_set_tunables(dg, update_mode=update_mode)
    for r in graphgen.pick_roots(g, 4, seed=22):
        check_root(g, dg, int(r))


def test_levels_deterministic_across_runs():
    g = graphgen.rmat(16, 16, seed=11)
    dg = load(g)
    r = int(graphgen.pick_roots(g, 1, seed=12)[0])
    first, _, _ = gpu_run(dg, r)
    for _ in range(5):
        lv, pa, _ = gpu_run(dg, r)
        assert np.array_equal(lv, first)


def test_host_output_and_async_stream():
    torch = torch_mod()
    g = graphgen.rmat(12, 16, seed=13)
    dg = load(g)
    r = int(graphgen.pick_roots(g, 1, seed=14)[0])
    ref, _, _ = oracle.bfs(g.offsets, g.cols, r)
    lv = np.empty(g.n, dtype=np.int32)
    pa = np.empty(g.n, dtype=np.int32)
    bfs.bfs_run(dg, r, lv, pa)  # BFS_OUT_HOST
    assert oracle.validate(g.offsets, g.cols, r, ref, lv, pa)[0] == 0
    s = torch.cuda.Stream()
    lvd = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pad = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(s):
        assert bfs.bfs_run(dg, r, lvd, pad, stream=s, flags=bfs.BFS_ASYNC) is None
    s.synchronize()
    assert oracle.validate(g.offsets, g.cols, r, ref, lvd.cpu().numpy(), pad.cpu().numpy())[0] == 0


def test_run_errors():
    torch = torch_mod()
    g = graphgen.path(10)
    dg = load(g)
    lv = torch.empty(10, dtype=torch.int32, device="cuda")
    for bad in (-1, 10):
        with pytest.raises(bfs.BfsError) as e:
            bfs.bfs_run(dg, bad, lv, lv)
        assert e.value.status == bfs.BFS_E_ROOT_RANGE
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run(dg, 0, lv, lv, flags=bfs.BFS_ASYNC | 0x80)
    assert e.value.status == bfs.BFS_E_INVALID_ARG


def test_rmat_scale20_64_roots():
    """R-MAT scale 20, edgefactor 16, int64 offsets, the 64 seeded roots."""
    g = graphgen.cached("rmat", scale=20, edgefactor=16, seed=1)
    dg = load(g)
    for r in graphgen.pick_roots(g, 64, seed=2):
        check_root(g, dg, int(r))


@pytest.mark.parametrize("tun", [dict(hot_vertices=8192, block_size=1024), dict(hot_vertices=8192, update_mode=2),
                                 dict(hot_vertices=16384, block_size=1024), dict(hot_vertices=16384, update_mode=2),
                                 dict(lds_visited=1, block_size=1024), dict(lds_visited=-1)])
def test_hot_bitmap_scale18(tun):
    """The LDS copy of the hot bitmap changes probes only, never results: levels
    exact and parents valid with the hot set on, for several roots."""
    g = graphgen.rmat(18, 16, seed=11)
    dg = load(g)
    bfs.bfs_graph_set_tunables(dg, **tun)
    for r in graphgen.pick_roots(g, 4, seed=12):
        check_root(g, dg, int(r))


def test_lds_visited_defaults_and_limit():
    """The whole visited bitmap goes to LDS by default from 2^16 to 2^20
    vertices (with 1024-thread workgroups); asking for it where the bitmap
    cannot fit is an argument error."""
    small = load(graphgen.rmat(15, 8, seed=31))
    assert bfs.bfs_graph_get_tunables(small)["lds_visited"] == -1
    mid = load(graphgen.rmat(17, 8, seed=32))
    t = bfs.bfs_graph_get_tunables(mid)
    assert (t["lds_visited"], t["block_size"]) == (1, 1024)
    t = bfs.bfs_graph_set_tunables(mid, block_size=256)
    assert t["lds_visited"] == -1  # the default follows the workgroup size
    big = load(graphgen.path((1 << 21) + 1))
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_graph_set_tunables(big, lds_visited=1, block_size=1024)
    assert e.value.status == bfs.BFS_E_INVALID_ARG


@pytest.mark.parametrize("sparse", [-1, 0, 3, 100])
def test_small_level_kernel_shapes(sparse):
    """Long chains of small levels (paths, a cycle, a binary tree, a star whose
    leaves all land in one restore block's list, a broom: a path into a big
    star, and a path, a star of 3000 leaves, then another path: small levels
    run in one workgroup twice with grid levels between, so the level offset
    they leave to later steps grows twice) give the same levels and valid
    parents with the small-level path off, at its default, and at tight limits."""
    two_tails = graphgen.from_edges(3201, list(range(50)) + [50] * 3000 + [3050] + list(range(3051, 3200)),
                                    list(range(1, 51)) + list(range(51, 3051)) + [3051] + list(range(3052, 3201)))
    cases = [(graphgen.path(3000), 0), (graphgen.path(3000), 1500), (graphgen.cycle(2001), 5),
             (graphgen.binary_tree(1 << 13), 0), (graphgen.star(5000), 0), (graphgen.star(5000), 17),
             (graphgen.from_edges(3000, list(range(999)) + [999] * 2000, list(range(1, 1000)) + list(range(1000, 3000))), 0),
             (two_tails, 0)]
    for g, r in cases:
        dg = load(g)
        bfs.bfs_graph_set_tunables(dg, sparse_frontier=sparse)
        check_root(g, dg, r)


@pytest.mark.parametrize("hot", [1500, 4096, 100000])
@pytest.mark.parametrize("flags", [0, bfs.BFS_HYBRID])
def test_hot_layout_ragged_vertex_count(hot, flags):
    """Hot sets on a skewed graph whose vertex count is not a multiple of 32
    (n = 50,001, 1562 full visited words): 1500 rounds up to 1536, one hot
    vertex per word; 4096 is capped at 3072, two per word (bits 0 and 16);
    100000 is capped the same way. Levels exact, parents valid, top-down and
    direction-optimising."""
    n = 50_001
    src, dst = graphgen.rmat_edges(16, 16 << 16, seed=61)
    g = graphgen.from_edges(n, (src % n).tolist(), (dst % n).tolist())
    dg = load(g, symmetric=True)
    bfs.bfs_graph_set_tunables(dg, hot_vertices=hot, block_size=1024)
    deg = np.diff(g.offsets)
    roots = [int(np.argmax(deg)), int(n - 1) if deg[n - 1] > 0 else int(np.flatnonzero(deg)[-1])]
    roots += [int(r) for r in graphgen.pick_roots(g, 2, seed=62)]
    for r in roots:
        check_root(g, dg, r, flags=flags)


@pytest.mark.parametrize("flags", [0, bfs.BFS_HYBRID])
def test_depth_changes_between_runs(flags):
    """Roots of very different depths, alternately, on one workspace of a graph
    with the degree-ordered copy: a run deeper than the previous one outlives
    the first chunk of levels, which already wrote its outputs and stop event,
    and must write both again at its end. Levels exact, parents valid, and a
    positive time every run."""
    g = graphgen.disjoint(graphgen.rmat(14, 16, seed=63), graphgen.path(300))
    dg = load(g, symmetric=True)
    bfs.bfs_graph_set_tunables(dg, hot_vertices=512, block_size=1024)
    shallow = int(graphgen.pick_roots(graphgen.rmat(14, 16, seed=63), 1, seed=64)[0])
    deep = g.n - 1  # one end of the path: 299 levels below it
    for r in (shallow, deep, shallow, shallow, deep, deep, shallow):
        _, _, st = check_root(g, dg, r, flags=flags)
        assert st["device_ms"] > 0.0
