"""The validator accepts every valid BFS tree and rejects mutated outputs (V1-V4)."""
import numpy as np
import pytest

import graphgen
import oracle
from tests import pins


@pytest.fixture(scope="module")
def case():
    g = graphgen.rmat(10, seed=1)
    r = int(graphgen.pick_roots(g, 1, seed=2)[0])
    lv, pa, _ = oracle.bfs(g.offsets, g.cols, r)
    return g, r, lv, pa


def test_accepts_oracle(case):
    g, r, lv, pa = case
    assert oracle.validate(g.offsets, g.cols, r, lv, lv, pa) == (0, -1)


def test_accepts_other_valid_parent():
    race = pins.load_golden("paper_examples.json")["benign_race"]
    g = graphgen.from_edges(race["n"], *zip(*race["edges"]))
    lv, pa, _ = oracle.bfs(g.offsets, g.cols, race["root"])
    for p in race["valid_parents"]:
        alt = pa.copy()
        alt[race["vertex"]] = p
        assert oracle.validate(g.offsets, g.cols, race["root"], lv, lv, alt)[0] == 0


def test_rejects_mutations(case):
    g, r, lv, pa = case
    reached = np.nonzero((lv > 0))[0]
    v = int(reached[len(reached) // 2])
    # V1: shifted level
    m = lv.copy(); m[v] += 1
    assert oracle.validate(g.offsets, g.cols, r, lv, m, pa)[0] == 1
    # V1: dropped reached vertex
    m = lv.copy(); m[v] = -1
    p = pa.copy(); p[v] = -1
    assert oracle.validate(g.offsets, g.cols, r, lv, m, p)[0] == 1
    # V2: root not its own parent
    p = pa.copy(); p[r] = int(g.cols[g.offsets[r]])
    assert oracle.validate(g.offsets, g.cols, r, lv, lv, p)[0] == 2
    # V3: reached vertex without parent
    p = pa.copy(); p[v] = -1
    assert oracle.validate(g.offsets, g.cols, r, lv, lv, p)[0] == 3
    # V4: parent at the same level / not adjacent / out of range
    same = np.nonzero(lv == lv[v])[0]
    p = pa.copy(); p[v] = int(same[same != v][0])
    assert oracle.validate(g.offsets, g.cols, r, lv, lv, p)[0] == 4
    up = np.nonzero(lv == lv[v] - 1)[0]
    row = set(g.cols[g.offsets[v]:g.offsets[v + 1]].tolist())
    nonadj = [u for u in up.tolist() if u not in row]
    if nonadj:
        p = pa.copy(); p[v] = nonadj[0]
        assert oracle.validate(g.offsets, g.cols, r, lv, lv, p) == (4, v)
    p = pa.copy(); p[v] = g.n + 3
    assert oracle.validate(g.offsets, g.cols, r, lv, lv, p)[0] == 4


def test_certify_accepts_valid_and_rejects_mutations(case):
    """V2-V5 without oracle levels accept exactly the hop distances."""
    g, r, lv, pa = case
    assert oracle.certify(g.offsets, g.cols, r, lv, pa) == (0, -1)
    reached = np.nonzero(lv > 0)[0]
    v = int(reached[len(reached) // 2])
    m = lv.copy(); m[v] += 1          # too far: its parent is no longer one level up
    assert oracle.certify(g.offsets, g.cols, r, m, pa)[0] in (4, 5)
    m = lv.copy(); m[v] -= 1          # too close
    assert oracle.certify(g.offsets, g.cols, r, m, pa)[0] in (4, 5)
    m = lv.copy(); p = pa.copy(); m[v] = -1; p[v] = -1   # dropped reached vertex
    assert oracle.certify(g.offsets, g.cols, r, m, p)[0] in (4, 5)
    m = np.where(lv > 0, lv * 2, lv).astype(np.int32)   # every level doubled
    assert oracle.certify(g.offsets, g.cols, r, m, pa)[0] != 0


def test_certify_agrees_with_validate_on_small_graphs():
    rng = np.random.default_rng(17)
    for _ in range(60):
        n = int(rng.integers(2, 40))
        g = graphgen.from_edges(n, rng.integers(0, n, 3 * n), rng.integers(0, n, 3 * n))
        r = int(rng.integers(0, n))
        lv, pa, _ = oracle.bfs(g.offsets, g.cols, r)
        assert oracle.certify(g.offsets, g.cols, r, lv, pa)[0] == 0
        if lv.max() >= 1:
            m = lv.copy()
            far = lv == lv.max()
            m[far] = lv.max() + 1     # the deepest layer pushed one level further
            assert oracle.certify(g.offsets, g.cols, r, m, pa)[0] != 0


def test_certify_rejects_level0_vertex_under_unreached_parent():
    """Directed graph 0->1, 2->3 from root 0: a second level-0 vertex whose
    'parent' is unreached must not pass (its parent chain never reaches the root)."""
    g = graphgen.from_edges(4, [0, 2], [1, 3], symmetric=False)
    lv = np.array([0, 1, -1, 0], dtype=np.int32)
    pa = np.array([0, 0, -1, 2], dtype=np.int32)
    assert oracle.certify(g.offsets, g.cols, 0, lv, pa) == (4, 3)
    ref, _, _ = oracle.bfs(g.offsets, g.cols, 0)
    assert ref.tolist() == [0, 1, -1, -1]
    assert oracle.validate(g.offsets, g.cols, 0, ref, lv, pa)[0] == 1


def test_checkers_accept_exactly_the_correct_candidates():
    """Exhaustive over every digraph on 3 vertices and every candidate output,
    plus single planted changes on random graphs (see tests/pins.py)."""
    lib = oracle._load()
    assert pins.pin_checkers_exhaustive(lib) == []
    assert pins.pin_checkers_planted(lib) == []
    assert pins.pin_checkers_directed_counterexample(lib) == []
