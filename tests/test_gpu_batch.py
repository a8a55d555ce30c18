"""GPU parity of batched multi-source BFS (bfs_run_batch through the C ABI):
every root's row has the oracle's levels and a valid BFS tree."""
import numpy as np
import pytest

import graphgen
import oracle
import paper_1604_02844_amd as bfs
from tests import pins
from tests.gpu_helpers import load, torch_mod

pytestmark = pytest.mark.gpu


def run_batch(dg, roots):
    torch = torch_mod()
    roots = np.asarray(roots, dtype=np.int32)
    lv = torch.empty((len(roots), dg.n), dtype=torch.int32, device="cuda")
    pa = torch.empty((len(roots), dg.n), dtype=torch.int32, device="cuda")
    st = bfs.bfs_run_batch(dg, roots, lv, pa)
    return lv.cpu().numpy(), pa.cpu().numpy(), st


def check_batch(g, dg, roots, rows_sorted=True):
    print(f"[case] bfs_run_batch {g.name} n={g.n} roots={len(roots)}", flush=True)
    lv, pa, st = run_batch(dg, roots)
    reached = arcs = 0
    for i, r in enumerate(roots):
        ref, _, ost = oracle.bfs(g.offsets, g.cols, int(r))
        code, bad = oracle.validate(g.offsets, g.cols, int(r), ref, lv[i], pa[i], rows_sorted=rows_sorted)
        assert code == 0, f"{g.name} slot {i} root {r}: {oracle.CHECK_NAMES[code]} at {bad}"
        reached += ost["reached"]
        arcs += ost["arcs"]
    assert st["reached"] == reached and st["arcs_scanned"] == arcs, (st, reached, arcs)
    assert st["num_roots"] == len(roots)
    return lv, pa, st


def test_closed_forms_batch():
    for g, r, exp_lv, _ in pins.closed_form_cases():
        roots = [r, 0, g.n - 1, r]  # includes a duplicate root
        check_batch(g, load(g), roots)


@pytest.mark.parametrize("width", [1, 8, 31, 32, 33, 63, 64, 65, 128])
def test_uneven_batch_widths(width):
    g = graphgen.rmat(12, 16, seed=31)
    roots = graphgen.pick_roots(g, width, seed=32)
    if len(roots) < width:  # repeat roots to reach the width
        roots = np.resize(roots, width)
    check_batch(g, load(g), roots)


def test_duplicate_and_isolated_roots():
    g = graphgen.disjoint(graphgen.rmat(10, 16, seed=33), graphgen.empty(5))
    roots = [g.n - 1, 3, 3, g.n - 2, 7]
    check_batch(g, load(g), roots)


@pytest.mark.parametrize("kind", ["rmat", "er"])
def test_batch_matches_single_root(kind):
    g = graphgen.rmat(14, 16, seed=34) if kind == "rmat" else graphgen.er(1 << 14, 16, seed=35)
    dg = load(g)
    roots = graphgen.pick_roots(g, 40, seed=36)
    lv, pa, _ = check_batch(g, dg, roots)
    torch = torch_mod()
    one_l = torch.empty(g.n, dtype=torch.int32, device="cuda")
    one_p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for i in (0, 17, 39):
        bfs.bfs_run(dg, int(roots[i]), one_l, one_p)
        assert np.array_equal(one_l.cpu().numpy(), lv[i])


@pytest.mark.parametrize("tun", [dict(small_max_degree=1, wave_max_degree=1), dict(wave_max_degree=100000),
                                 dict(batch_width=7), dict(batch_width=64, blocks_per_cu=1)])
def test_batch_tunables(tun):
    g = graphgen.rmat(13, 16, seed=37)
    dg = load(g)
    bfs.bfs_graph_set_tunables(dg, **tun)
    check_batch(g, dg, graphgen.pick_roots(g, 20, seed=38))


def test_unreached_fill_and_final_pass():
    """Unreached (root, vertex) pairs get -1 from a fill before the batch (the
    first batch on a workspace, or after one that left many pairs unreached)
    or from a pass after it that writes only those pairs (after a batch that
    reached nearly every pair). On one workspace: a batch in a large connected
    component (fill; 0.6% of pairs unreached), one confined to a 50-vertex path
    (pass, with nearly every pair unreached), the same again (fill), then the
    large component twice (fill, then pass). Outputs start as uninitialised
    memory, so a pair written by neither shows up. Every row exact."""
    big = graphgen.er(1 << 13, 16, seed=91)
    g = graphgen.disjoint(big, graphgen.path(50))
    dg = load(g)
    roots_big = graphgen.pick_roots(big, 32, seed=92)
    roots_small = [big.n + 3, big.n + 10, big.n + 49]
    for roots in (roots_big, roots_small, roots_small, roots_big, roots_big):
        check_batch(g, dg, roots)
    # Host outputs (staging rows) after a batch that chose the pass.
    lv = np.empty((len(roots_big), g.n), dtype=np.int32)
    pa = np.empty((len(roots_big), g.n), dtype=np.int32)
    bfs.bfs_run_batch(dg, roots_big, lv, pa)
    for i, r in enumerate(roots_big):
        ref, _, _ = oracle.bfs(g.offsets, g.cols, int(r))
        assert oracle.validate(g.offsets, g.cols, int(r), ref, lv[i], pa[i])[0] == 0


def test_batch_int32_offsets_and_host_output():
    g = graphgen.rmat(10, 16, seed=1)
    dg = load(g, offsets_i32=True)
    roots = graphgen.pick_roots(g, 16, seed=2)
    lv = np.empty((len(roots), g.n), dtype=np.int32)
    pa = np.empty((len(roots), g.n), dtype=np.int32)
    bfs.bfs_run_batch(dg, roots, lv, pa)  # host buffers: BFS_OUT_HOST
    for i, r in enumerate(roots):
        ref, _, _ = oracle.bfs(g.offsets, g.cols, int(r))
        assert oracle.validate(g.offsets, g.cols, int(r), ref, lv[i], pa[i])[0] == 0


def test_batch_errors():
    g = graphgen.path(10)
    dg = load(g)
    torch = torch_mod()
    lv = torch.empty((2, 10), dtype=torch.int32, device="cuda")
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run_batch(dg, [0, 10], lv, lv)
    assert e.value.status == bfs.BFS_E_ROOT_RANGE
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run_batch(dg, np.zeros(0, dtype=np.int32), lv, lv)
    assert e.value.status == bfs.BFS_E_INVALID_ARG


def test_er_batches_8_32_64():
    """Uniform random graph (2^16 vertices, average degree 16), batches of 8, 32, 64."""
    g = graphgen.er(1 << 16, 16, seed=39)
    dg = load(g)
    pool = graphgen.pick_roots(g, 64, seed=40)
    for b in (8, 32, 64):
        check_batch(g, dg, pool[:b])


def test_pull_long_rows():
    """Dense levels where rows longer than a lane's head are scanned by the
    whole wavefront: a star whose hub is reached from 64 leaf roots, a complete
    graph, two hubs joined by a path (the scan must run past early windows
    that find nothing), and R-MAT with 64 roots."""
    star = graphgen.star(5000)
    check_batch(star, load(star), list(range(1, 65)))
    comp = graphgen.complete(300)
    check_batch(comp, load(comp), list(range(0, 300, 5))[:64])
    n = 6000
    src = [0] * 2000 + [5999] * 2000 + list(range(2000, 3999))
    dst = list(range(1, 2001)) + list(range(3000, 5000)) + list(range(2001, 4000))
    broom = graphgen.from_edges(n, src, dst)
    check_batch(broom, load(broom), [1, 2, 3, 4999, 4998, 2500, 3500, 0, 5999])
    g = graphgen.rmat(16, 16, seed=39)
    check_batch(g, load(g), graphgen.pick_roots(g, 64, seed=40))


@pytest.mark.parametrize("persistent", [1, -1])
@pytest.mark.parametrize("case", ["rmat14", "path", "widths"])
def test_persistent_and_per_level_launches(persistent, case):
    """Both launch forms of a batch: one cooperative launch running every level
    behind grid barriers, and one launch per kernel and level (the default).
    Levels identical to the oracle, parents valid, totals equal; a deep graph
    (a 3000-vertex path: 3000 levels in one launch) and uneven widths."""
    if case == "rmat14":
        g = graphgen.rmat(14, 16, seed=91)
        roots = graphgen.pick_roots(g, 64, seed=92)
    elif case == "path":
        g = graphgen.disjoint(graphgen.path(3000), graphgen.star(50))
        roots = [0, 1500, 2999, 3000, 3010]
    else:
        g = graphgen.er(1 << 13, 6, seed=93)
        roots = np.resize(graphgen.pick_roots(g, 40, seed=94), 97)
    dg = load(g)
    bfs.bfs_graph_set_tunables(dg, persistent=persistent)
    assert bfs.bfs_graph_get_tunables(dg)["persistent"] == persistent
    check_batch(g, dg, roots)
    bfs.bfs_graph_free(dg)
