"""Pins of the oracle's deterministic predecessors (least in-neighbour one level
up): closed forms of path, cycle, complete graph, star, grid and binary tree,
every labelled graph on 4 vertices against matrix-power distances, and random
digraphs with self-loops and duplicates against Bellman-Ford distances."""
import numpy as np
import pytest

import graphgen
import oracle
from tests import pins


def test_min_parent_pins_hold():
    assert pins.pin_min_parents(oracle._load()) == []


def test_min_parents_form_a_valid_tree():
    g = graphgen.rmat(12, 8, seed=41)
    for r in graphgen.pick_roots(g, 4, seed=42):
        lv, _, _ = oracle.bfs(g.offsets, g.cols, int(r))
        pa = oracle.min_parents(g.offsets, g.cols, int(r), lv)
        assert oracle.validate(g.offsets, g.cols, int(r), lv, lv, pa)[0] == 0


def test_min_parents_reject_a_wrong_level_array():
    g = graphgen.path(10)
    lv, _, _ = oracle.bfs(g.offsets, g.cols, 0)
    lv = lv.copy()
    lv[5] = 7  # no neighbour at level 6
    with pytest.raises(ValueError):
        oracle.min_parents(g.offsets, g.cols, 0, lv)
