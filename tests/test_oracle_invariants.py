"""Invariants of BFS that hold at any size, checked on generated graphs."""
import numpy as np
import pytest

import graphgen
import oracle
from tests import pins


@pytest.mark.parametrize("kind", ["rmat", "er"])
def test_invariants_generated(kind):
    g = graphgen.rmat(11, seed=5) if kind == "rmat" else graphgen.er(3000, 3.0, seed=6)
    roots = graphgen.pick_roots(g, 4, seed=9)
    deg = g.degrees()
    src = np.repeat(np.arange(g.n), deg)
    for r in roots:
        lv, pa, st = oracle.bfs(g.offsets, g.cols, int(r))
        comp = pins.union_find_component(g.n, g.offsets, g.cols, int(r))
        assert np.array_equal(lv >= 0, comp)                       # reached set == component
        both = (lv[src] >= 0)
        assert np.all(lv[g.cols][both] >= 0)                       # arcs from reached reach reached
        assert np.all(np.abs(lv[src][both] - lv[g.cols][both]) <= 1)  # symmetric: |dl| <= 1
        assert np.bincount(lv[lv >= 0]).sum() == st["reached"]
        assert st["arcs"] == int(deg[lv >= 0].sum())
        assert st["levels"] == int(lv.max()) + 1
        assert np.all(np.bincount(lv[lv >= 0]) > 0)                # layers are contiguous
        assert oracle.validate(g.offsets, g.cols, int(r), lv, lv, pa)[0] == 0


def test_table1_shape_scale20():
    """Section 4.1 / Table 1 as a shape: ~7 layers, two layers with >98% of arcs, ~60% reached."""
    t1 = pins.load_golden("paper_examples.json")["table1_shape"]
    g = graphgen.rmat(20, seed=1)
    roots = graphgen.pick_roots(g, 3, seed=2)
    for r in roots:
        lv, _, st = oracle.bfs(g.offsets, g.cols, int(r))
        deg = g.degrees()
        per_layer = np.bincount(lv[lv >= 0], weights=deg[lv >= 0])
        top2 = np.sort(per_layer)[-2:].sum() / per_layer.sum()
        assert 5 <= st["levels"] <= 10
        assert top2 > 0.95 and abs(top2 - t1["top_two_share"]) < 0.05
        assert 0.5 < st["reached"] / g.n < 0.75
        assert abs(st["reached"] - t1["reached_approx"]) / t1["reached_approx"] < 0.1
