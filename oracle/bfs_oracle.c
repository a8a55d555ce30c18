/*
 * CPU oracle for top-down BFS — TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library. The GPU product path never calls it and shares no
 * code with it: no headers, no helpers, no tables.
 *
 * What it computes (plain C, int32 / int64 integers, no floating point):
 *
 *   oracle_bfs       The textbook serial FIFO-queue BFS (paper section 3: a
 *                    queue with constant-time enqueue/dequeue, O(V+E)), written
 *                    in the shape of the serial top-down algorithm (section 3.1,
 *                    Algorithm 1): every vertex starts with no predecessor, the
 *                    source is its own predecessor, each dequeued vertex scans
 *                    its whole neighbour list and every not-yet-visited
 *                    neighbour is marked visited, recorded with the dequeued
 *                    vertex as predecessor and queued.
 *                    levels[v] is the layer index of v (section 3: a layer is
 *                    the set of vertices at the same distance from the source,
 *                    distance counted in edges); unreached vertices get -1 in
 *                    both arrays (the paper's "infinity" predecessor, read as -1).
 *                    Because levels[] is a hop distance it is unique, so the GPU
 *                    path must reproduce it exactly. parents[] is not unique
 *                    (section 3.2: different correct BFS trees can result), so
 *                    the oracle's FIFO-first parent is never compared directly;
 *                    oracle_validate checks a candidate tree instead.
 *
 *   oracle_validate  Complete check of a candidate (levels, parents) against the
 *                    oracle's levels: V1 levels identical; V2 root is level 0 and
 *                    its own parent; V3 level -1 exactly where parent -1; V4 every
 *                    other reached vertex has a parent in range, one level up,
 *                    joined to it by an arc parent -> vertex.
 *
 *   oracle_certify   The same verdict without running a BFS, for outputs too
 *                    large to recompute one by one: V2-V4 plus V5, every arc
 *                    u -> v leaving a reached u reaches v with
 *                    levels[v] <= levels[u] + 1. V4 asks every reached vertex
 *                    other than the root for a level of at least 1 and a
 *                    parent one level lower; following parents therefore
 *                    lowers the level by one per arc until it reaches level 0,
 *                    which only the root holds (V2 and V4), so every reached v
 *                    has a walk of levels[v] arcs from the root and
 *                    levels[v] >= its hop distance. V5 applied along a shortest
 *                    path from the root shows every vertex on it reached with
 *                    levels[v] <= its hop distance. Hence V2-V5 hold exactly
 *                    when levels[] is the hop distance (-1 where unreachable)
 *                    and parents[] a BFS tree, on directed graphs as well.
 *
 *   oracle_min_parents  Deterministic predecessors. Any reached neighbour one
 *                    layer up is a correct predecessor (section 3.2), so the
 *                    smallest one is a unique choice: for every reached v other
 *                    than the root, the least u with an arc u -> v and
 *                    levels[u] = levels[v] - 1. Written as that definition, one
 *                    pass over every arc taking minima; it needs only levels[]
 *                    (any correct level array, e.g. oracle_bfs's).
 *
 * Pins: tests/test_oracle_*.py check this file against brute force on every
 * labelled graph with n <= 6, unit-weight Bellman-Ford on random digraphs,
 * closed forms (path, cycle, star, complete graph, grid, binary tree, disjoint
 * components) and the paper's worked examples. The two checkers are pinned by
 * tests/test_validator.py: over every digraph on 3 vertices they accept exactly
 * the candidate outputs (all levels and parents in -1..2) that equal the
 * matrix-power distances and pass a pure-Python tree check, and on random
 * directed and symmetric graphs they judge every single planted change of a
 * level or a parent as that check does. Planted mistakes in copies of this
 * file (tests/test_oracle_mutants.py) must each fail one of these pins.
 */
#include <stdint.h>
#include <stdlib.h>

enum { ORACLE_OK = 0, ORACLE_E_ARG = -1, ORACLE_E_ROOT = -3, ORACLE_E_MEM = -4, ORACLE_E_LEVELS = -5 };

/*
 * stats (nullable) receives: [0] R reached vertices, [1] A arcs scanned
 * (sum of out-degrees of reached vertices), [2] L number of non-empty layers.
 */
int oracle_bfs(int64_t n, const int64_t* offsets, const int32_t* cols, int64_t root,
               int32_t* levels, int32_t* parents, int64_t* stats) {
    if (n < 1 || !offsets || !levels || !parents) return ORACLE_E_ARG;
    if (root < 0 || root >= n) return ORACLE_E_ROOT;

    int32_t* queue = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!queue) return ORACLE_E_MEM;

    for (int64_t v = 0; v < n; ++v) {
        levels[v] = -1;
        parents[v] = -1;
    }
    levels[root] = 0;
    parents[root] = (int32_t)root;
    int64_t head = 0, tail = 0;
    queue[tail++] = (int32_t)root;

    int64_t arcs = 0;
    while (head < tail) {
        int32_t u = queue[head++];
        int64_t begin = offsets[u], end = offsets[u + 1];
        arcs += end - begin;
        for (int64_t j = begin; j < end; ++j) {
            int32_t v = cols[j];
            if (levels[v] == -1) { /* not visited */
                levels[v] = levels[u] + 1;
                parents[v] = u;
                queue[tail++] = v;
            }
        }
    }
    if (stats) {
        stats[0] = tail;
        stats[1] = arcs;
        stats[2] = (int64_t)levels[queue[tail - 1]] + 1;
    }
    free(queue);
    return ORACLE_OK;
}

/* Does row u contain v? Binary search when rows are sorted, else a scan. */
static int has_arc(const int64_t* offsets, const int32_t* cols, int64_t u, int32_t v, int sorted) {
    int64_t lo = offsets[u], hi = offsets[u + 1];
    if (!sorted) {
        for (int64_t j = lo; j < hi; ++j)
            if (cols[j] == v) return 1;
        return 0;
    }
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cols[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < offsets[u + 1] && cols[lo] == v;
}

/* V2-V4 of a candidate against its own levels (shared by both checks). V4
 * includes the level bound: a reached vertex other than the root sits at
 * level 1 or deeper, so its parent is itself reached. */
static int check_tree(int64_t n, const int64_t* offsets, const int32_t* cols, int64_t root,
                      const int32_t* levels, const int32_t* parents, int rows_sorted,
                      int64_t* bad_vertex) {
    if (levels[root] != 0 || parents[root] != root) { /* V2 */
        if (bad_vertex) *bad_vertex = root;
        return 2;
    }
    for (int64_t v = 0; v < n; ++v) { /* V3 */
        if ((levels[v] == -1) != (parents[v] == -1)) {
            if (bad_vertex) *bad_vertex = v;
            return 3;
        }
    }
    for (int64_t v = 0; v < n; ++v) { /* V4 */
        if (v == root || levels[v] == -1) continue;
        int64_t u = parents[v];
        if (levels[v] < 1 || u < 0 || u >= n || levels[u] != levels[v] - 1 ||
            !has_arc(offsets, cols, u, (int32_t)v, rows_sorted)) {
            if (bad_vertex) *bad_vertex = v;
            return 4;
        }
    }
    return 0;
}

/*
 * Returns 0 when the candidate passes V1-V4, otherwise the number (1..4) of the
 * first failing check; *bad_vertex (nullable) receives the offending vertex.
 * Negative returns are argument errors.
 */
int oracle_validate(int64_t n, const int64_t* offsets, const int32_t* cols, int64_t root,
                    const int32_t* ref_levels, const int32_t* levels, const int32_t* parents,
                    int rows_sorted, int64_t* bad_vertex) {
    if (n < 1 || !offsets || !ref_levels || !levels || !parents) return ORACLE_E_ARG;
    if (root < 0 || root >= n) return ORACLE_E_ROOT;
    if (bad_vertex) *bad_vertex = -1;
    for (int64_t v = 0; v < n; ++v) { /* V1 */
        if (levels[v] != ref_levels[v]) {
            if (bad_vertex) *bad_vertex = v;
            return 1;
        }
    }
    return check_tree(n, offsets, cols, root, levels, parents, rows_sorted, bad_vertex);
}

/*
 * V2-V5 without oracle levels (see the header). Returns 0 or the failing check
 * number (2..5); negative on argument errors.
 */
int oracle_certify(int64_t n, const int64_t* offsets, const int32_t* cols, int64_t root,
                   const int32_t* levels, const int32_t* parents, int rows_sorted, int64_t* bad_vertex) {
    if (n < 1 || !offsets || !levels || !parents) return ORACLE_E_ARG;
    if (root < 0 || root >= n) return ORACLE_E_ROOT;
    if (bad_vertex) *bad_vertex = -1;
    for (int64_t v = 0; v < n; ++v) {
        if (levels[v] < -1 || levels[v] >= n) {
            if (bad_vertex) *bad_vertex = v;
            return 3;
        }
    }
    int rc = check_tree(n, offsets, cols, root, levels, parents, rows_sorted, bad_vertex);
    if (rc) return rc;
    for (int64_t u = 0; u < n; ++u) { /* V5 */
        if (levels[u] == -1) continue;
        for (int64_t j = offsets[u]; j < offsets[u + 1]; ++j) {
            int32_t v = cols[j];
            if (levels[v] == -1 || levels[v] > levels[u] + 1) {
                if (bad_vertex) *bad_vertex = v;
                return 5;
            }
        }
    }
    return 0;
}

/*
 * parents[v] = the least in-neighbour of v one level up, for every reached v
 * other than the root; parents[root] = root; -1 where levels[v] = -1.
 * Returns ORACLE_E_LEVELS (and *bad_vertex) if a reached vertex other than the
 * root has no such in-neighbour, i.e. levels[] is not a BFS level array.
 */
int oracle_min_parents(int64_t n, const int64_t* offsets, const int32_t* cols, int64_t root,
                       const int32_t* levels, int32_t* parents, int64_t* bad_vertex) {
    if (n < 1 || !offsets || !levels || !parents) return ORACLE_E_ARG;
    if (root < 0 || root >= n) return ORACLE_E_ROOT;
    if (bad_vertex) *bad_vertex = -1;
    for (int64_t v = 0; v < n; ++v) parents[v] = levels[v] < 0 ? -1 : INT32_MAX;
    parents[root] = (int32_t)root;
    for (int64_t u = 0; u < n; ++u) {
        if (levels[u] < 0) continue;
        for (int64_t j = offsets[u]; j < offsets[u + 1]; ++j) {
            const int32_t v = cols[j];
            if (levels[v] != levels[u] + 1) continue;  /* the root (level 0) never qualifies */
            if (u < parents[v]) parents[v] = (int32_t)u;
        }
    }
    for (int64_t v = 0; v < n; ++v) {
        if (parents[v] == INT32_MAX) {
            if (bad_vertex) *bad_vertex = v;
            return ORACLE_E_LEVELS;
        }
    }
    return ORACLE_OK;
}
