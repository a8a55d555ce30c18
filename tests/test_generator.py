"""The seeded input generators: R-MAT statistics, CSR invariants, determinism."""
import numpy as np
import pytest

import graphgen


def _csr_invariants(g):
    off, col = g.offsets, g.cols
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == len(col)
    assert col.dtype == np.int32 and (len(col) == 0 or (col.min() >= 0 and col.max() < g.n))
    src = np.repeat(np.arange(g.n), np.diff(off))
    assert not np.any(src == col)                                  # no self-loops
    key = src.astype(np.int64) * g.n + col
    assert np.all(np.diff(key) > 0)                                # rows sorted, no duplicates
    rev = np.sort(col.astype(np.int64) * g.n + src)
    assert np.array_equal(rev, key)                                # symmetric


@pytest.mark.parametrize("scale", [6, 10, 14])
def test_rmat_csr_invariants(scale):
    _csr_invariants(graphgen.rmat(scale, seed=3))


def test_er_csr_invariants():
    _csr_invariants(graphgen.er(5000, 8, seed=4))


def test_rmat_quadrant_frequencies():
    """Top-level quadrant of each raw draw follows A, B, C, D (chi-square, 3 dof)."""
    scale, m = 12, 200_000
    src, dst = graphgen.rmat_edges(scale, m, seed=7)
    top = 1 << (scale - 1)
    q = (src >= top) * 2 + (dst >= top)
    counts = np.bincount(q, minlength=4)
    exp = m * np.array([0.57, 0.19, 0.19, 0.05])
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 16.3  # p = 0.001 for 3 degrees of freedom
    # every bit level, not only the top one
    for lvl in range(scale):
        b = 1 << lvl
        ql = ((src & b) > 0) * 2 + ((dst & b) > 0)
        c = np.bincount(ql, minlength=4)
        assert ((c - exp) ** 2 / exp).sum() < 20


def test_rmat_edge_count_and_determinism():
    g1 = graphgen.rmat(12, seed=5)
    g2 = graphgen.rmat(12, seed=5)
    g3 = graphgen.rmat(12, seed=6)
    assert np.array_equal(g1.offsets, g2.offsets) and np.array_equal(g1.cols, g2.cols)
    assert not np.array_equal(g1.cols[:100], g3.cols[:100]) or g1.nnz != g3.nnz
    assert g1.nnz <= 2 * 16 * (1 << 12)
    assert g1.nnz > 0.6 * 2 * 16 * (1 << 12)


def test_permutation_is_bijection_and_relabels():
    p = graphgen.permutation(1 << 12, 9)
    assert np.array_equal(np.sort(p), np.arange(1 << 12))
    raw = graphgen.rmat(12, seed=5, perm_seed=-1)
    rel = graphgen.rmat(12, seed=5)
    assert raw.nnz == rel.nnz
    assert np.array_equal(np.sort(raw.degrees()), np.sort(rel.degrees()))
    # unpermuted R-MAT concentrates degree on low ids; relabelling spreads it
    assert raw.degrees()[:64].sum() > 5 * rel.degrees()[:64].sum()


def test_pick_roots():
    g = graphgen.rmat(10, seed=1)
    r = graphgen.pick_roots(g, 16, seed=2)
    assert len(r) == 16 and len(set(r.tolist())) == 16
    assert np.all(g.degrees()[r] > 0)
    assert np.array_equal(r, graphgen.pick_roots(g, 16, seed=2))
    tiny = graphgen.disjoint(graphgen.path(3), graphgen.empty(5))
    assert sorted(graphgen.pick_roots(tiny, 10, seed=1).tolist()) == [0, 1, 2]


def test_closed_form_shapes():
    assert graphgen.path(5).nnz == 8
    assert graphgen.cycle(5).nnz == 10
    assert graphgen.star(5).nnz == 8
    assert graphgen.complete(6).nnz == 30
    assert graphgen.grid(3, 4).nnz == 2 * (3 * 3 + 2 * 4)
    assert graphgen.binary_tree(7).nnz == 12
    for g in (graphgen.path(50), graphgen.grid(7, 9), graphgen.binary_tree(63), graphgen.complete(9)):
        _csr_invariants(g)
