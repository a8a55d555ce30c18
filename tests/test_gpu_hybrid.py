"""GPU parity of direction-optimising runs (BFS_HYBRID): levels with large
frontiers run bottom-up. Levels must equal the oracle's exactly, parents must
be valid, and reached / arcs_scanned / num_levels must equal the top-down
definition, on graphs whose frontiers switch direction several times."""
import numpy as np
import pytest

import graphgen
import oracle
import paper_1604_02844_amd as bfs
from tests.gpu_helpers import check_root, load, torch_mod

pytestmark = pytest.mark.gpu
H = bfs.BFS_HYBRID


def test_hybrid_closed_forms():
    torch_mod()
    cases = [graphgen.path(3000), graphgen.cycle(2001), graphgen.star(5000), graphgen.complete(200),
             graphgen.grid(80, 120), graphgen.binary_tree(1 << 14),
             graphgen.disjoint(graphgen.grid(30, 30), graphgen.star(300))]
    for g in cases:
        dg = load(g, symmetric=True)
        for r in (0, g.n // 2, g.n - 1):
            check_root(g, dg, r, flags=H)


@pytest.mark.parametrize("scale", [10, 14, 18])
def test_hybrid_rmat(scale):
    g = graphgen.rmat(scale, 16, seed=21)
    dg = load(g, symmetric=True)
    for r in graphgen.pick_roots(g, 4, seed=22):
        check_root(g, dg, int(r), flags=H)


def test_hybrid_erdos_renyi_and_int32_offsets():
    g = graphgen.er(1 << 16, 8, seed=23)
    dg = load(g, offsets_i32=True, symmetric=True)
    for r in graphgen.pick_roots(g, 3, seed=24):
        check_root(g, dg, int(r), flags=H)


@pytest.mark.parametrize("tun", [dict(update_mode=2), dict(hot_vertices=8192, block_size=1024),
                                 dict(hot_vertices=16384, block_size=1024),
                                 dict(small_max_degree=1, wave_max_degree=1),
                                 dict(lds_visited=1, block_size=1024), dict(lds_visited=-1)])
def test_hybrid_tunables(tun):
    g = graphgen.rmat(18, 16, seed=25)
    dg = load(g, symmetric=True)
    bfs.bfs_graph_set_tunables(dg, **tun)
    for r in graphgen.pick_roots(g, 3, seed=26):
        check_root(g, dg, int(r), flags=H)


def test_hybrid_same_levels_as_top_down():
    g = graphgen.rmat(16, 16, seed=27)
    dg = load(g, symmetric=True)
    for r in graphgen.pick_roots(g, 3, seed=28):
        lv_td, _, st_td = check_root(g, dg, int(r))
        lv_h, _, st_h = check_root(g, dg, int(r), flags=H)
        assert np.array_equal(lv_td, lv_h)
        assert (st_td["reached"], st_td["arcs_scanned"], st_td["num_levels"]) == \
               (st_h["reached"], st_h["arcs_scanned"], st_h["num_levels"])


def test_hybrid_errors():
    torch = torch_mod()
    g = graphgen.rmat(10, 16, seed=29)
    dg = load(g)  # not declared symmetric
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty_like(lv)
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run(dg, 0, lv, pa, flags=H)
    assert e.value.status == bfs.BFS_E_INVALID_ARG
    # a directed graph declared symmetric is rejected at load
    d = graphgen.from_edges(8, [0, 1, 2], [1, 2, 3], symmetric=False)
    with pytest.raises(bfs.BfsError) as e:
        load(d, symmetric=True)
    assert e.value.status == bfs.BFS_E_INVALID_GRAPH
