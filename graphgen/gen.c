/*
 * Seeded synthetic graph generators (host C, OpenMP).
 *
 * This module produces the input graphs that both the GPU BFS library and the
 * CPU oracle consume. It holds none of the BFS arithmetic: it only draws edges,
 * relabels vertices and assembles a symmetric, deduplicated CSR.
 *
 * Families:
 *   - R-MAT / Kronecker (the paper's workload, section "Input graph" and the
 *     "Which layers are vectorized?" subsection): 2^S vertices, ef * 2^S drawn
 *     edges, one quadrant draw per bit level with initiator (A, B, C, D).
 *   - Erdos-Renyi G(n, M): M uniform vertex pairs.
 *
 * Shared conventions (readings where the paper is silent):
 *   - counter-based RNG: the SplitMix64 finaliser applied to key + ctr * golden;
 *     every edge is a pure function of (seed, edge index), so the two CSR passes
 *     regenerate the same edges without storing an edge list;
 *   - no noise on the initiator: exact A, B, C, D at every bit level;
 *   - vertex ids are relabelled with a seeded Fisher-Yates permutation;
 *   - every undirected pair {a, b}, a != b, gives arcs a->b and b->a; self
 *     loops are dropped; duplicate arcs are removed; rows are sorted ascending.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GOLDEN 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* One 64-bit draw for stream `key` at position `ctr`. */
static inline uint64_t rng_at(uint64_t key, uint64_t ctr) {
    return mix64(key + (ctr + 1) * GOLDEN);
}

static inline double rng_unit(uint64_t key, uint64_t ctr) {
    return (double)(rng_at(key, ctr) >> 11) * (1.0 / 9007199254740992.0);
}

/* Uniform integer in [0, bound) by a 64x64 -> high-64 multiply. */
static inline uint64_t rng_below(uint64_t key, uint64_t ctr, uint64_t bound) {
    return (uint64_t)(((unsigned __int128)rng_at(key, ctr) * bound) >> 64);
}

static uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return mix64(seed * 0xd1b54a32d192ed03ULL + stream * GOLDEN + 0x632be59bd9b4e019ULL);
}

int gg_version(void) { return 1; }

/* Seeded random permutation of [0, n): Fisher-Yates driven by rng_below. */
int gg_permutation(int64_t n, uint64_t seed, int32_t* perm) {
    if (n < 0 || !perm) return -1;
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    uint64_t key = stream_key(seed, 7);
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)rng_below(key, (uint64_t)i, (uint64_t)(i + 1));
        int32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Edge sources. An edge source maps an edge index e to an (a, b) pair.
 * ------------------------------------------------------------------------- */
typedef struct {
    int kind; /* 0 = R-MAT, 1 = Erdos-Renyi */
    int scale;
    int64_t n;
    uint64_t key;
    double ab, abc, a; /* cumulative initiator thresholds */
    const int32_t* perm; /* may be NULL */
} edge_src;

static inline void edge_at(const edge_src* s, int64_t e, int64_t* pa, int64_t* pb) {
    int64_t a = 0, b = 0;
    if (s->kind == 0) {
        uint64_t base = (uint64_t)e * 64u;
        for (int l = 0; l < s->scale; ++l) {
            double u = rng_unit(s->key, base + (uint64_t)l);
            int64_t bit = (int64_t)1 << (s->scale - 1 - l);
            if (u < s->a) {
                /* quadrant A: (0, 0) */
            } else if (u < s->ab) {
                b |= bit; /* quadrant B: (0, 1) */
            } else if (u < s->abc) {
                a |= bit; /* quadrant C: (1, 0) */
            } else {
                a |= bit; /* quadrant D: (1, 1) */
                b |= bit;
            }
        }
    } else {
        a = (int64_t)rng_below(s->key, 2 * (uint64_t)e, (uint64_t)s->n);
        b = (int64_t)rng_below(s->key, 2 * (uint64_t)e + 1, (uint64_t)s->n);
    }
    if (s->perm) {
        a = s->perm[a];
        b = s->perm[b];
    }
    *pa = a;
    *pb = b;
}

static int cmp_i32(const void* x, const void* y) {
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

/* Insertion sort for short rows, qsort for long ones. */
static void sort_row(int32_t* r, int64_t len) {
    if (len < 32) {
        for (int64_t i = 1; i < len; ++i) {
            int32_t x = r[i];
            int64_t j = i - 1;
            while (j >= 0 && r[j] > x) {
                r[j + 1] = r[j];
                --j;
            }
            r[j + 1] = x;
        }
    } else {
        qsort(r, (size_t)len, sizeof(int32_t), cmp_i32);
    }
}

/*
 * Build the symmetric deduplicated CSR of `m` edges from `src`.
 * offsets: int64[n+1] (caller-allocated). cols: int32[2*m] (caller-allocated;
 * the first offsets[n] entries hold the result). Returns nnz or < 0 on error.
 */
static int64_t build_csr(const edge_src* src, int64_t n, int64_t m, int nthreads,
                         int64_t* offsets, int32_t* cols) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!deg) return -2;

    /* Pass 1: degrees before deduplication. */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        int64_t a, b;
        edge_at(src, e, &a, &b);
        if (a == b) continue;
#pragma omp atomic
        deg[a]++;
#pragma omp atomic
        deg[b]++;
    }
    /* Exclusive prefix sum into offsets; deg becomes the fill cursor. */
    offsets[0] = 0;
    for (int64_t v = 0; v < n; ++v) offsets[v + 1] = offsets[v] + deg[v];
    for (int64_t v = 0; v < n; ++v) deg[v] = offsets[v];

    /* Pass 2: fill rows (order inside a row is fixed by the sort below). */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        int64_t a, b;
        edge_at(src, e, &a, &b);
        if (a == b) continue;
        int64_t pa, pb;
#pragma omp atomic capture
        pa = deg[a]++;
#pragma omp atomic capture
        pb = deg[b]++;
        cols[pa] = (int32_t)b;
        cols[pb] = (int32_t)a;
    }

    /* Sort and deduplicate each row in place; deg[v] becomes the new length. */
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; ++v) {
        int32_t* r = cols + offsets[v];
        int64_t len = offsets[v + 1] - offsets[v];
        sort_row(r, len);
        int64_t k = 0;
        for (int64_t i = 0; i < len; ++i)
            if (k == 0 || r[i] != r[k - 1]) r[k++] = r[i];
        deg[v] = k;
    }

    /* Compact rows to the left, in row order (new start <= old start). */
    int64_t pos = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t old = offsets[v];
        int64_t len = deg[v];
        if (pos != old && len) memmove(cols + pos, cols + old, (size_t)len * sizeof(int32_t));
        offsets[v] = pos;
        pos += len;
    }
    offsets[n] = pos;
    free(deg);
    return pos;
}

/*
 * R-MAT graph with 2^scale vertices and m = edgefactor * 2^scale drawn edges.
 * cols must hold 2*m int32 entries. perm_seed < 0 disables relabelling.
 */
int64_t gg_rmat(int scale, int64_t edgefactor, double A, double B, double C, uint64_t seed,
                int64_t perm_seed, int nthreads, int64_t* offsets, int32_t* cols) {
    if (scale < 1 || scale > 30 || edgefactor < 1 || !offsets || !cols) return -1;
    if (!(A >= 0 && B >= 0 && C >= 0 && A + B + C <= 1.0)) return -1;
    int64_t n = (int64_t)1 << scale;
    int64_t m = edgefactor * n;
    int32_t* perm = NULL;
    if (perm_seed >= 0) {
        perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
        if (!perm) return -2;
        gg_permutation(n, (uint64_t)perm_seed, perm);
    }
    edge_src s;
    memset(&s, 0, sizeof s);
    s.kind = 0;
    s.scale = scale;
    s.n = n;
    s.key = stream_key(seed, 1);
    s.a = A;
    s.ab = A + B;
    s.abc = A + B + C;
    s.perm = perm;
    int64_t nnz = build_csr(&s, n, m, nthreads, offsets, cols);
    free(perm);
    return nnz;
}

/* Erdos-Renyi G(n, M) with m uniform pairs. cols must hold 2*m entries. */
int64_t gg_er(int64_t n, int64_t m, uint64_t seed, int nthreads, int64_t* offsets, int32_t* cols) {
    if (n < 1 || n > 2147483647LL || m < 0 || !offsets || !cols) return -1;
    edge_src s;
    memset(&s, 0, sizeof s);
    s.kind = 1;
    s.n = n;
    s.key = stream_key(seed, 2);
    return build_csr(&s, n, m, nthreads, offsets, cols);
}

/* Raw (undeduplicated, unpermuted) R-MAT edge draws, for statistical tests. */
int gg_rmat_edges(int scale, double A, double B, double C, uint64_t seed, int64_t e0, int64_t count,
                  int64_t* src, int64_t* dst) {
    if (scale < 1 || scale > 30 || !src || !dst) return -1;
    edge_src s;
    memset(&s, 0, sizeof s);
    s.kind = 0;
    s.scale = scale;
    s.n = (int64_t)1 << scale;
    s.key = stream_key(seed, 1);
    s.a = A;
    s.ab = A + B;
    s.abc = A + B + C;
    for (int64_t i = 0; i < count; ++i) edge_at(&s, e0 + i, &src[i], &dst[i]);
    return 0;
}

/*
 * Distinct roots of degree > 0, drawn in a fixed seeded order (rejection of
 * repeats and of isolated vertices). Returns the number drawn (< k if the
 * graph has fewer than k non-isolated vertices).
 */
int64_t gg_pick_roots(int64_t n, const int64_t* offsets, int64_t k, uint64_t seed, int32_t* out) {
    if (n < 1 || !offsets || !out || k < 0) return -1;
    int64_t eligible = 0;
    for (int64_t v = 0; v < n; ++v) eligible += offsets[v + 1] > offsets[v];
    if (k > eligible) k = eligible;
    uint8_t* taken = (uint8_t*)calloc((size_t)n, 1);
    if (!taken) return -2;
    uint64_t key = stream_key(seed, 3);
    int64_t got = 0;
    for (uint64_t ctr = 0; got < k; ++ctr) {
        int64_t v = (int64_t)rng_below(key, ctr, (uint64_t)n);
        if (taken[v] || offsets[v + 1] == offsets[v]) continue;
        taken[v] = 1;
        out[got++] = (int32_t)v;
    }
    free(taken);
    return got;
}

/* Uniform draws in [0, bound), for serving traces (graph choice, roots, gaps). */
int gg_uniform_u64(uint64_t seed, uint64_t stream, int64_t count, uint64_t bound, uint64_t* out) {
    if (!out || count < 0) return -1;
    uint64_t key = stream_key(seed, 100 + stream);
    for (int64_t i = 0; i < count; ++i)
        out[i] = bound ? rng_below(key, (uint64_t)i, bound) : rng_at(key, (uint64_t)i);
    return 0;
}

int gg_uniform_f64(uint64_t seed, uint64_t stream, int64_t count, double* out) {
    if (!out || count < 0) return -1;
    uint64_t key = stream_key(seed, 200 + stream);
    for (int64_t i = 0; i < count; ++i) out[i] = rng_unit(key, (uint64_t)i);
    return 0;
}
