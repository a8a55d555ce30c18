"""Independent checks that pin the CPU oracle (and, through it, the GPU path).

Every function here takes the oracle's ctypes library handle so that the same
checks can be re-run against deliberately mutated copies of the oracle source
(``test_oracle_mutants.py``): a pin set that lets a plausible mistake through is
itself a test failure.

Nothing here re-types the oracle's loop. The references are of other kinds:
boolean adjacency-matrix powers, unit-weight Bellman-Ford, closed-form distance
formulas, and values printed in the paper (``tests/golden/``).
"""
from __future__ import annotations

import json
import os

import numpy as np

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name: str):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# Brute-force references
# ---------------------------------------------------------------------------

def all_graph_adjacency(n: int) -> np.ndarray:
    """Adjacency matrices of every labelled simple undirected graph on n vertices."""
    iu, ju = np.triu_indices(n, 1)
    k = len(iu)
    masks = np.arange(1 << k, dtype=np.int64)
    bits = ((masks[:, None] >> np.arange(k)) & 1).astype(bool)
    adj = np.zeros((1 << k, n, n), dtype=bool)
    adj[:, iu, ju] = bits
    adj[:, ju, iu] = bits
    return adj


def matrix_power_levels(adj: np.ndarray) -> np.ndarray:
    """dist[g, r, v] = least k with (A^k)[r, v] > 0, else -1 (boolean matrix powers)."""
    g, n, _ = adj.shape
    a = adj.astype(np.int64)
    dist = np.full((g, n, n), -1, dtype=np.int64)
    reach = np.broadcast_to(np.eye(n, dtype=np.int64), (g, n, n)).copy()  # A^0
    for k in range(n):
        newly = (reach > 0) & (dist == -1)
        dist[newly] = k
        reach = np.minimum(reach @ a, 1)
    return dist


def bellman_ford_levels(n: int, src, dst, root: int) -> np.ndarray:
    """Unit-weight Bellman-Ford over an arc list: relax every arc n-1 times."""
    INF = 1 << 40
    d = [INF] * n
    d[root] = 0
    for _ in range(max(n - 1, 1)):
        changed = False
        for a, b in zip(src, dst):
            if d[a] + 1 < d[b]:
                d[b] = d[a] + 1
                changed = True
        if not changed:
            break
    return np.array([x if x < INF else -1 for x in d], dtype=np.int64)


def union_find_component(n: int, offsets, cols, root: int) -> np.ndarray:
    """Boolean mask of root's component (undirected reading) by union-find."""
    parent = np.arange(n)

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    deg = np.diff(offsets)
    src = np.repeat(np.arange(n), deg)
    for a, b in zip(src.tolist(), np.asarray(cols).tolist()):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    r = find(root)
    return np.array([find(v) == r for v in range(n)])


def check_parents_python(n, offsets, cols, root, levels, parents) -> bool:
    """Independent (pure-Python) statement of V2-V4 for small graphs."""
    if levels[root] != 0 or parents[root] != root:
        return False
    for v in range(n):
        if (levels[v] == -1) != (parents[v] == -1):
            return False
        if v == root or levels[v] == -1:
            continue
        u = int(parents[v])
        if not (0 <= u < n) or levels[u] != levels[v] - 1:
            return False
        if v not in set(cols[offsets[u]:offsets[u + 1]].tolist()):
            return False
    return True


# ---------------------------------------------------------------------------
# Pin sets (each returns a list of failure strings; empty = pinned)
# ---------------------------------------------------------------------------

def pin_exhaustive(lib, n: int) -> list[str]:
    """Every labelled simple graph on n vertices, every root, vs matrix powers."""
    adj = all_graph_adjacency(n)
    dist = matrix_power_levels(adj)
    fails = []
    for gi in range(adj.shape[0]):
        rows, cols = np.nonzero(adj[gi])
        offsets = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(np.bincount(rows, minlength=n), out=offsets[1:])
        cols = cols.astype(np.int32)
        for r in range(n):
            lv, pa, _ = oracle.bfs(offsets, cols, r, lib=lib)
            if not np.array_equal(lv, dist[gi, r]):
                fails.append(f"n={n} graph={gi} root={r}: levels {lv.tolist()} != {dist[gi, r].tolist()}")
            elif not check_parents_python(n, offsets, cols, r, lv, pa):
                fails.append(f"n={n} graph={gi} root={r}: invalid parents {pa.tolist()}")
            if len(fails) > 5:
                return fails
    return fails


def closed_form_cases():
    """(graph, root, expected levels, expected unique parents or None)."""
    cases = []
    n = 1000
    v = np.arange(n)
    for r in (0, 377, n - 1):
        exp_par = np.where(v < r, v + 1, v - 1)
        exp_par[r] = r
        cases.append((graphgen.path(n), r, np.abs(v - r), exp_par))
    for cn in (999, 1000):
        r = 17
        d = np.abs(v[:cn] - r)
        cases.append((graphgen.cycle(cn), r, np.minimum(d, cn - d), None))
    cases.append((graphgen.star(500), 0, np.r_[0, np.ones(499, dtype=np.int64)],
                  np.zeros(500, dtype=np.int64)))
    lv = np.full(500, 2)
    lv[7], lv[0] = 0, 1
    par = np.zeros(500, dtype=np.int64)
    par[7], par[0] = 7, 7
    cases.append((graphgen.star(500), 7, lv, par))
    lv = np.ones(60, dtype=np.int64)
    lv[11] = 0
    cases.append((graphgen.complete(60), 11, lv, np.full(60, 11)))
    R, C = 37, 53
    rr, cc = np.divmod(np.arange(R * C), C)
    root = 20 * C + 9
    cases.append((graphgen.grid(R, C), root, np.abs(rr - 20) + np.abs(cc - 9), None))
    nb = 4095
    vb = np.arange(nb)
    par = (vb - 1) // 2
    par[0] = 0
    cases.append((graphgen.binary_tree(nb), 0, np.floor(np.log2(vb + 1)).astype(np.int64), par))
    g2 = graphgen.disjoint(graphgen.path(10), graphgen.complete(5))
    lv = np.r_[np.arange(10), np.full(5, -1)]
    cases.append((g2, 0, lv, np.r_[0, np.arange(9), np.full(5, -1)]))
    g3 = graphgen.disjoint(graphgen.empty(1), graphgen.star(6))
    cases.append((g3, 0, np.r_[0, np.full(6, -1)], np.r_[0, np.full(6, -1)]))
    return cases


def pin_closed_forms(lib) -> list[str]:
    fails = []
    for g, r, exp_lv, exp_par in closed_form_cases():
        lv, pa, st = oracle.bfs(g.offsets, g.cols, r, lib=lib)
        if not np.array_equal(lv, exp_lv):
            bad = np.nonzero(lv != exp_lv)[0][:5]
            fails.append(f"{g.name} root {r}: levels differ at {bad.tolist()}")
            continue
        if exp_par is not None and not np.array_equal(pa, exp_par):
            fails.append(f"{g.name} root {r}: parents differ")
        reached = int((exp_lv >= 0).sum())
        if st["reached"] != reached or st["levels"] != int(exp_lv.max()) + 1:
            fails.append(f"{g.name} root {r}: stats {st}")
        if st["arcs"] != int(g.degrees()[exp_lv >= 0].sum()):
            fails.append(f"{g.name} root {r}: arc count {st['arcs']}")
    return fails


def pin_paper_examples(lib) -> list[str]:
    fails = []
    ex = load_golden("paper_examples.json")
    race = ex["benign_race"]
    g = graphgen.from_edges(race["n"], *zip(*race["edges"]))
    lv, pa, _ = oracle.bfs(g.offsets, g.cols, race["root"], lib=lib)
    for v, lev in race["levels"].items():
        if lv[int(v)] != lev:
            fails.append(f"benign race: level[{v}]={lv[int(v)]} expected {lev}")
    if int(pa[race["vertex"]]) not in race["valid_parents"]:
        fails.append(f"benign race: parent {pa[race['vertex']]} not in {race['valid_parents']}")
    word = ex["bit_race_word"]
    g = graphgen.from_edges(word["n"], [word["root"]] * len(word["children"]), word["children"])
    lv, pa, _ = oracle.bfs(g.offsets, g.cols, word["root"], lib=lib)
    if not all(lv[c] == 1 and pa[c] == word["root"] for c in word["children"]):
        fails.append("bit-race word: a child of the root was lost")
    return fails


def pin_bellman_ford(lib, n, src, dst, root) -> list[str]:
    g = graphgen.from_edges(n, src, dst, symmetric=False, dedupe=False, drop_self_loops=False,
                            sort_rows=False)
    lv, pa, _ = oracle.bfs(g.offsets, g.cols, root, lib=lib)
    ref = bellman_ford_levels(n, src, dst, root)
    if not np.array_equal(lv, ref):
        return [f"bellman-ford mismatch n={n} root={root}"]
    if not check_parents_python(n, g.offsets, g.cols, root, lv, pa):
        return [f"invalid parents n={n} root={root}"]
    return []


def pin_random_digraphs(lib, count: int = 60, seed: int = 11) -> list[str]:
    rng = np.random.default_rng(seed)
    fails = []
    for _ in range(count):
        n = int(rng.integers(1, 48))
        m = int(rng.integers(0, 4 * n))
        src = rng.integers(0, n, m)
        dst = rng.integers(0, n, m)
        fails += pin_bellman_ford(lib, n, src.tolist(), dst.tolist(), int(rng.integers(0, n)))
    return fails


# ---------------------------------------------------------------------------
# Deterministic predecessors (least in-neighbour one level up)
# ---------------------------------------------------------------------------

def _min_parent_reference(n, src, dst, dist, root) -> np.ndarray:
    """From reference distances: least u over arcs u -> v with dist[u] = dist[v] - 1."""
    ref = np.where(dist >= 0, np.iinfo(np.int32).max, -1).astype(np.int64)
    for u, v in zip(src, dst):
        if v != root and dist[u] >= 0 and dist[v] == dist[u] + 1:
            ref[v] = min(ref[v], u)
    ref[root] = root
    return ref


def min_parent_closed_forms():
    """(graph, root, expected least parents) from the shape of the graph alone."""
    cases = []
    n = 1000
    v = np.arange(n)
    for r in (0, 377, n - 1):
        exp = np.where(v < r, v + 1, v - 1)
        exp[r] = r
        cases.append((graphgen.path(n), r, exp))
    # Cycle: the vertex opposite the root (even length) has two parents, the
    # neighbours on either side; the least is the smaller id.
    for cn, r in ((1000, 0), (1000, 17), (999, 17)):
        u = np.arange(cn)
        d = (u - r) % cn
        fwd = np.where(d <= cn // 2, (u - 1) % cn, (u + 1) % cn)  # one step back along the shorter way
        exp = fwd.copy()
        if cn % 2 == 0:
            opp = (r + cn // 2) % cn
            exp[opp] = min((opp - 1) % cn, (opp + 1) % cn)
        exp[r] = r
        cases.append((graphgen.cycle(cn), r, exp))
    cases.append((graphgen.complete(60), 11, np.full(60, 11)))
    exp = np.zeros(500, dtype=np.int64)  # star centre 0: every leaf hangs off it ...
    exp[0] = exp[7] = 7                     # ... except leaf 7, the root, which is the centre's parent
    cases.append((graphgen.star(500), 7, exp))
    # Grid: the neighbours one step closer to the root are (i -/+ 1, j) and
    # (i, j -/+ 1) toward it; ids are i * C + j, so the row step is the smaller
    # id exactly when it moves up a row.
    R, C = 37, 53
    ri, cj = 20, 9
    rr, cc = np.divmod(np.arange(R * C), C)
    cand = np.full(R * C, np.iinfo(np.int64).max)
    up = rr > ri
    down = rr < ri
    left = cc > cj
    right = cc < cj
    cand = np.where(up, np.minimum(cand, (rr - 1) * C + cc), cand)
    cand = np.where(down, np.minimum(cand, (rr + 1) * C + cc), cand)
    cand = np.where(left, np.minimum(cand, rr * C + cc - 1), cand)
    cand = np.where(right, np.minimum(cand, rr * C + cc + 1), cand)
    cand[ri * C + cj] = ri * C + cj
    cases.append((graphgen.grid(R, C), ri * C + cj, cand))
    nb = 4095
    par = (np.arange(nb) - 1) // 2
    par[0] = 0
    cases.append((graphgen.binary_tree(nb), 0, par))
    return cases


def pin_min_parents(lib) -> list[str]:
    fails = []
    for g, r, exp in min_parent_closed_forms():
        lv, _, _ = oracle.bfs(g.offsets, g.cols, r, lib=lib)
        try:
            pa = oracle.min_parents(g.offsets, g.cols, r, lv, lib=lib)
        except ValueError as e:
            fails.append(f"{g.name} root {r}: {e}")
            continue
        if not np.array_equal(pa, exp):
            bad = np.nonzero(pa != exp)[0][:5]
            fails.append(f"{g.name} root {r}: least parents differ at {bad.tolist()}")
    # Every labelled simple graph on 4 vertices, every root, against matrix-power distances.
    n = 4
    adj = all_graph_adjacency(n)
    dist = matrix_power_levels(adj)
    for gi in range(adj.shape[0]):
        src, dst = np.nonzero(adj[gi])
        offsets = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(np.bincount(src, minlength=n), out=offsets[1:])
        for r in range(n):
            ref = _min_parent_reference(n, src.tolist(), dst.tolist(), dist[gi, r], r)
            try:
                pa = oracle.min_parents(offsets, dst.astype(np.int32), r, dist[gi, r], lib=lib)
            except ValueError as e:
                fails.append(f"exhaustive n=4 graph {gi} root {r}: {e}")
                continue
            if not np.array_equal(pa, ref):
                fails.append(f"exhaustive n=4 graph {gi} root {r}: {pa.tolist()} != {ref.tolist()}")
            if len(fails) > 5:
                return fails
    # Random digraphs with self-loops and duplicates, against Bellman-Ford distances.
    rng = np.random.default_rng(19)
    for _ in range(20):
        n = int(rng.integers(1, 40))
        m = int(rng.integers(0, 4 * n))
        src = rng.integers(0, n, m).tolist()
        dst = rng.integers(0, n, m).tolist()
        r = int(rng.integers(0, n))
        g = graphgen.from_edges(n, src, dst, symmetric=False, dedupe=False, drop_self_loops=False,
                                sort_rows=False)
        dist = bellman_ford_levels(n, src, dst, r)
        ref = _min_parent_reference(n, src, dst, dist, r)
        try:
            pa = oracle.min_parents(g.offsets, g.cols, r, dist, lib=lib)
        except ValueError as e:
            fails.append(f"digraph n={n} root {r}: {e}")
            continue
        if not np.array_equal(pa, ref):
            fails.append(f"digraph n={n} root {r}: least parents differ")
    return fails


# ---------------------------------------------------------------------------
# The checkers themselves (validate: V1-V4 against reference levels; certify:
# V2-V5 on its own). A candidate is correct exactly when its levels are the hop
# distances and its parents a BFS tree (the paper's section 3.2: any discoverer
# one layer up is a correct predecessor); both checkers must accept exactly the
# correct candidates.
# ---------------------------------------------------------------------------

def all_digraph_adjacency(n: int) -> np.ndarray:
    """Adjacency matrices of every labelled digraph on n vertices without self-loops."""
    off = [(i, j) for i in range(n) for j in range(n) if i != j]
    k = len(off)
    masks = np.arange(1 << k, dtype=np.int64)
    bits = ((masks[:, None] >> np.arange(k)) & 1).astype(bool)
    adj = np.zeros((1 << k, n, n), dtype=bool)
    adj[:, [a for a, _ in off], [b for _, b in off]] = bits
    return adj


def _checker_calls(lib, n, offsets, cols, root, ref, rows_sorted):
    """Two callables (validate, certify) taking candidate arrays written in place
    into fixed buffers: one ctypes call per candidate, no conversions."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    col = np.ascontiguousarray(cols, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    rl = np.ascontiguousarray(ref, dtype=np.int32)
    lv = np.zeros(n, dtype=np.int32)
    pa = np.zeros(n, dtype=np.int32)
    bad = np.zeros(1, dtype=np.int64)
    po, pc, pr, pl, pp, pb = (a.ctypes.data for a in (off, col, rl, lv, pa, bad))
    srt = int(bool(rows_sorted))

    def validate(levels, parents):
        lv[:] = levels
        pa[:] = parents
        return lib.oracle_validate(n, po, pc, root, pr, pl, pp, srt, pb)

    def certify(levels, parents):
        lv[:] = levels
        pa[:] = parents
        return lib.oracle_certify(n, po, pc, root, pl, pp, srt, pb)

    return validate, certify


def pin_checkers_exhaustive(lib, n: int = 3) -> list[str]:
    """Every labelled digraph on n vertices (root 0: relabelling covers the other
    roots), every candidate with levels and parents in {-1, .., n-1}: validate
    (given the matrix-power distances) and certify both accept exactly the
    candidates whose levels equal those distances and whose parents pass the
    pure-Python tree check."""
    adj = all_digraph_adjacency(n)
    dist = matrix_power_levels(adj)
    vals = np.arange(-1, n)
    grid = np.array(np.meshgrid(*([vals] * n), indexing="ij")).reshape(n, -1).T  # all value vectors
    fails = []
    root = 0
    for gi in range(adj.shape[0]):
        src, dst = np.nonzero(adj[gi])
        offsets = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(np.bincount(src, minlength=n), out=offsets[1:])
        cols = dst.astype(np.int32)
        d = dist[gi, root]
        validate, certify = _checker_calls(lib, n, offsets, cols, root, d, True)
        for lvv in grid:
            same = np.array_equal(lvv, d)
            for pav in grid:
                truth = same and check_parents_python(n, offsets, cols, root, lvv, pav)
                if (validate(lvv, pav) == 0) != truth:
                    fails.append(f"validate digraph {gi} levels {lvv.tolist()} parents {pav.tolist()}: "
                                 f"{'rejected' if truth else 'accepted'}")
                if (certify(lvv, pav) == 0) != truth:
                    fails.append(f"certify digraph {gi} levels {lvv.tolist()} parents {pav.tolist()}: "
                                 f"{'rejected' if truth else 'accepted'}")
                if len(fails) > 5:
                    return fails
    return fails


def _python_parents(n, offsets, cols, dist, root, pick_max: bool):
    """A BFS tree from reference distances, chosen without the oracle: the
    largest (or smallest) in-neighbour one level up."""
    pa = np.full(n, -1, dtype=np.int64)
    for u in range(n):
        if dist[u] < 0:
            continue
        for v in cols[offsets[u]:offsets[u + 1]].tolist():
            if v != root and dist[v] == dist[u] + 1:
                if pa[v] < 0 or (u > pa[v] if pick_max else u < pa[v]):
                    pa[v] = u
    pa[root] = root
    return pa


def pin_checkers_planted(lib, count: int = 40, seed: int = 23) -> list[str]:
    """Random graphs (directed and symmetric, rows sorted, degrees up to ~12):
    a correct tree from Bellman-Ford distances is accepted by both checkers, and
    every single planted change of one level or one parent is judged as the
    pure-Python check judges it."""
    rng = np.random.default_rng(seed)
    fails = []
    for it in range(count):
        n = int(rng.integers(4, 24))
        m = int(rng.integers(n, 6 * n))
        src = rng.integers(0, n, m).tolist()
        dst = rng.integers(0, n, m).tolist()
        sym = bool(it % 2)
        g = graphgen.from_edges(n, src, dst, symmetric=sym)
        asrc = np.repeat(np.arange(n), np.diff(g.offsets)).tolist()
        root = int(rng.integers(0, n))
        dist = bellman_ford_levels(n, asrc, g.cols.tolist(), root)
        validate, certify = _checker_calls(lib, n, g.offsets, g.cols, root, dist, True)
        for pick_max in (False, True):
            pa = _python_parents(n, g.offsets, g.cols, dist, root, pick_max)
            if validate(dist, pa) != 0 or certify(dist, pa) != 0:
                fails.append(f"n={n} root={root}: a correct tree was rejected")
        base_pa = _python_parents(n, g.offsets, g.cols, dist, root, False)
        for v in range(n):
            for val in range(-1, n + 1):
                for which in ("level", "parent"):
                    lv = dist.copy()
                    pa = base_pa.copy()
                    if which == "level":
                        if val == lv[v]:
                            continue
                        lv[v] = val
                    else:
                        if val == pa[v]:
                            continue
                        pa[v] = val
                    truth = np.array_equal(lv, dist) and check_parents_python(n, g.offsets, g.cols, root, lv, pa)
                    if (validate(lv, pa) == 0) != truth or (certify(lv, pa) == 0) != truth:
                        fails.append(f"n={n} root={root} {which}[{v}]={val}: misjudged (correct={truth})")
                    if len(fails) > 5:
                        return fails
    return fails


def pin_checkers_directed_counterexample(lib) -> list[str]:
    """Digraph 0->1, 2->3 from root 0: vertex 3 claims level 0 through the
    unreached vertex 2. Both checkers must reject it."""
    g = graphgen.from_edges(4, [0, 2], [1, 3], symmetric=False)
    lv = np.array([0, 1, -1, 0])
    pa = np.array([0, 0, -1, 2])
    ref = np.array([0, 1, -1, -1])
    validate, certify = _checker_calls(lib, 4, g.offsets, g.cols, 0, ref, True)
    fails = []
    if certify(lv, pa) == 0:
        fails.append("certify accepts a second level-0 vertex under an unreached parent")
    if validate(lv, pa) == 0:
        fails.append("validate accepts a second level-0 vertex under an unreached parent")
    return fails
