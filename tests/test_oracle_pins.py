"""Pins of the CPU oracle against references that are not the oracle itself.

Brute force (boolean matrix powers over every labelled graph with n <= 6,
unit-weight Bellman-Ford on random digraphs with self-loops and duplicate arcs),
closed forms, and the paper's worked examples (tests/golden/paper_examples.json).
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import graphgen
import oracle
from tests import pins


@pytest.fixture(scope="module")
def lib():
    oracle.build()
    return oracle._load()


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_exhaustive_small_graphs(lib, n):
    fails = pins.pin_exhaustive(lib, n)
    assert not fails, fails


def test_closed_forms(lib):
    fails = pins.pin_closed_forms(lib)
    assert not fails, fails


def test_paper_examples(lib):
    fails = pins.pin_paper_examples(lib)
    assert not fails, fails


def test_random_digraphs_bellman_ford(lib):
    fails = pins.pin_random_digraphs(lib, count=80)
    assert not fails, fails


@settings(max_examples=150, deadline=None)
@given(st.integers(1, 40).flatmap(lambda n: st.tuples(
    st.just(n),
    st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=5 * n),
    st.integers(0, n - 1))))
def test_hypothesis_digraphs(data):
    n, arcs, root = data
    src = [a for a, _ in arcs]
    dst = [b for _, b in arcs]
    fails = pins.pin_bellman_ford(oracle._load(), n, src, dst, root)
    assert not fails, fails


def test_root_out_of_range(lib):
    g = graphgen.path(5)
    for r in (-1, 5, 1 << 40):
        with pytest.raises(ValueError):
            oracle.bfs(g.offsets, g.cols, r)


def test_self_loops_and_duplicates_do_not_change_levels(lib):
    rng = np.random.default_rng(3)
    n = 300
    src = rng.integers(0, n, 900)
    dst = rng.integers(0, n, 900)
    clean = graphgen.from_edges(n, src, dst)
    dirty = graphgen.from_edges(n, np.r_[src, src, np.arange(n)], np.r_[dst, dst, np.arange(n)],
                                dedupe=False, drop_self_loops=False)
    for r in (0, 5, 77):
        a, _, _ = oracle.bfs(clean.offsets, clean.cols, r)
        b, pb, _ = oracle.bfs(dirty.offsets, dirty.cols, r)
        assert np.array_equal(a, b)
        assert oracle.validate(dirty.offsets, dirty.cols, r, a, b, pb, rows_sorted=False)[0] == 0
