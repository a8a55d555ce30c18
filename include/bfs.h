/*
 * bfs.h — C ABI of libbfs.so: level-synchronous top-down breadth-first search
 * on one AMD Instinct MI355X (gfx950).
 *
 * The problem statement follows the paper (Paredes, Riley, Lujan, "Breadth
 * First Search Vectorization on the Intel Xeon Phi", arXiv 1604.02844):
 * section 3 — given a graph G and a source vertex s, explore every edge that
 * can be reached from s and output a BFS spanning tree as a predecessor list;
 * layers L_k hold the vertices at distance k (distance = number of edges on a
 * shortest path) and are processed in order; section 3.1, Algorithm 1 — every
 * vertex starts with no predecessor, the source is its own predecessor, and a
 * neighbour that is not yet visited is marked visited, put in the next layer
 * and given the expanding vertex as predecessor; section 3.3.1 — the graph is
 * stored as CSR and the visited / input / output sets are bitmaps of 32-bit
 * words (vertex v in word v/32, bit v%32).
 *
 * Output conventions (shared by every call that returns a BFS result):
 *   levels[v]  = hop distance from the root, or -1 when v is unreached
 *                (unique, so it is reproducible exactly);
 *   parents[v] = a vertex u with levels[u] == levels[v]-1 and an arc u->v;
 *                parents[root] = root; -1 when v is unreached. When several
 *                parents are valid any one may be returned (section 3.2: the
 *                parent race is benign and different correct BFS trees can
 *                result), so parents may differ between runs.
 *
 * General rules:
 *   - Every function returns an int status: BFS_OK (0), BFS_PENDING (1, poll
 *     only) or a negative BFS_E_* error. No C++ exception crosses this ABI.
 *   - Vertex ids are int32 (n <= 2^31-1); arc positions are int64.
 *   - Pointers are host pointers unless a flag says otherwise. "Device
 *     pointer" means memory from hipMalloc (or a torch CUDA tensor) on the
 *     device the library runs on.
 *   - A `stream` argument is a hipStream_t passed as void*; NULL means the
 *     default (null) stream.
 */
#ifndef BFS_H
#define BFS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define BFS_OK 0
#define BFS_PENDING 1              /* bfs_server_poll: request not finished yet */
#define BFS_E_INVALID_ARG (-1)     /* NULL pointer, bad size, bad flag combination */
#define BFS_E_INVALID_GRAPH (-2)   /* n<1, n>2^31-1, offsets[0]!=0, decreasing offsets,
                                      offsets[n]!=nnz, or a column outside [0,n) */
#define BFS_E_ROOT_RANGE (-3)      /* a root outside [0,n) */
#define BFS_E_NO_MEMORY (-4)       /* device or host allocation failed, or over budget */
#define BFS_E_DEVICE (-5)          /* a HIP runtime error */
#define BFS_E_UNKNOWN_TICKET (-6)  /* ticket never issued or already consumed */
#define BFS_E_BUSY (-7)            /* object still in use (e.g. graph held by a server) */
#define BFS_E_SHUTDOWN (-8)        /* server is shutting down */
#define BFS_E_INTERNAL (-9)        /* an unexpected internal failure */

/* ---- flags --------------------------------------------------------------- */
/* bfs_graph_load_csr */
#define BFS_LOAD_DEVICE_PTRS 0x1u   /* offsets/cols are device pointers, borrowed (not
                                       copied): they must outlive the graph */
#define BFS_LOAD_SKIP_VALIDATE 0x2u /* trust the CSR; skip the O(n+nnz) checks */
#define BFS_LOAD_OFFSETS_I32 0x4u   /* offsets points at int32_t[n+1] instead of int64_t[n+1];
                                       the graph keeps 4-byte offsets on the device */
#define BFS_LOAD_SYMMETRIC 0x8u     /* the CSR is symmetric (u->v present iff v->u, counted with
                                       multiplicity); checked at load unless SKIP_VALIDATE
                                       (BFS_E_INVALID_GRAPH if not). Needed by BFS_HYBRID. */
/* bfs_run / bfs_run_batch */
#define BFS_OUT_HOST 0x1u           /* levels/parents are host pointers (results are copied
                                       back before return; implies synchronous) */
#define BFS_ASYNC 0x2u              /* enqueue on `stream` and return; stats must be NULL */
#define BFS_HYBRID 0x4u             /* bfs_run only: a level whose frontier is large runs
                                       bottom-up (every unvisited vertex looks for a frontier
                                       neighbour) instead of top-down; same levels, valid
                                       parents. Requires a graph loaded with BFS_LOAD_SYMMETRIC. */
#define BFS_DETERMINISTIC 0x10u     /* bfs_run only: after the levels are final, every reached
                                       vertex other than the root gets the least in-neighbour one
                                       level up as parent (any such neighbour is correct, section
                                       3.2; the least is unique), so parents[] no longer depends on
                                       the timing of the run. Part of the timed run. */

typedef struct bfs_graph bfs_graph;
typedef struct bfs_server bfs_server;

/* Totals of one run (for a batch: summed over roots, num_levels = max). */
typedef struct {
    int32_t num_levels;      /* non-empty layers = max level + 1 */
    int32_t num_roots;       /* 1 for bfs_run */
    int64_t reached;         /* vertices with level >= 0 */
    int64_t arcs_scanned;    /* sum of out-degrees of reached vertices */
    int64_t edges_traversed; /* arcs_scanned / 2: undirected edges of the root's
                                component on a symmetric graph (the TEPS numerator) */
    double device_ms;        /* device time of the run (HIP events on `stream`) */
} bfs_run_stats;

/* Kernel tunables. Zero fields mean "library default". See bfs_autotune. */
typedef struct {
    int32_t small_max_degree;   /* T1: rows with d <= T1 are packed, several per wavefront */
    int32_t wave_max_degree;    /* T2: T1 < d <= T2 gets one wavefront; the arcs of all rows
                                   with d > T2 are split evenly over the whole grid */
    int32_t chunk_arcs;         /* fewest arcs of rows above T2 handed to one workgroup */
    int32_t blocks_per_cu;      /* workgroups per compute unit of the expansion grid */
    int32_t block_size;         /* threads per expansion workgroup: 256, 512 or 1024 */
    int32_t batch_width;        /* bfs_run_batch: roots per bit-sliced pass (1..64) */
    int32_t update_mode;        /* bitmap update: 1 = plain read-modify-write followed by the
                                   restoration pass (the paper's atomic-free scheme, section
                                   3.3.2), 2 = atomicOr claim; 0 = library default */
    int32_t hot_vertices;       /* single-root runs: every workgroup keeps the visited bits of
                                   this many vertices (the highest-degree ones, taken from a
                                   degree-ordered copy of the graph) in LDS during levels with
                                   large frontiers and probes them there first; rounded up to
                                   a multiple of 64 and capped at 2^20 and at two per full
                                   32-vertex word (one per word while they fit, else two);
                                   -1 = off, 0 = library default (2^20 from 2^22 vertices on
                                   skewed graphs) */
    int32_t lds_visited;        /* single-root runs without the degree-ordered copy: every
                                   workgroup copies the whole visited bitmap (bottom-up levels:
                                   the whole frontier bitmap) into LDS at the start of a level
                                   with a large frontier and probes it there first. 1 = on
                                   (BFS_E_INVALID_ARG from bfs_graph_set_tunables if the bitmap
                                   does not fit in LDS beside the workgroup), -1 = off, 0 =
                                   library default (on for 2^16..2^20 vertices, with 1024-thread
                                   workgroups) */
    int32_t sparse_frontier;    /* single-root runs: a level whose frontier has at most this
                                   many vertices (at most 4096) and at most 4 times as many arcs
                                   is expanded by the expansion kernel's first workgroup alone,
                                   from the list of the frontier the previous restoration made,
                                   with exact atomicOr claims; consecutive such levels run in
                                   that one launch. On, it reserves 80 KiB of the expansion's LDS
                                   (within the 128 KiB the hot bitmap takes by default; smaller
                                   workgroups without the hot bitmap then fit fewer per CU).
                                   -1 = off, 0 = library default (1024) */
    int32_t block_vertices;     /* single-root runs on the degree-ordered copy: rows above T2
                                   keep their arcs grouped by destination block of this many
                                   vertices (a power of two from 2^11 to 2^20, rounded down), and
                                   a level with a large frontier expands those rows block by
                                   block, each workgroup holding its block's visited bits in LDS
                                   (exact for earlier levels, so no probe leaves the workgroup
                                   for them); -1 = off, 0 = library default (off: slower
                                   at R-MAT scale 24, where a row's arcs split into short
                                   per-block runs) */
    int32_t persistent;         /* bfs_run_batch: 1 = every level of a group in one cooperative
                                   launch (grid-wide barriers between a level's expansion and its
                                   finish pass, the loop ending on the device at the first empty
                                   frontier); -1 = one launch per kernel and level, with a host
                                   check between chunks of levels; 0 = library default (-1:
                                   the cooperative kernel holds fewer waves per CU and is slower) */
    int32_t hub_bins;           /* single-root runs: at a level whose frontier is small but whose
                                   rows above T2 carry many arcs (the level that expands the hubs),
                                   each arc's head and parent go to a bin of its 8192-vertex
                                   destination chunk instead of probing the global visited
                                   bitmap; the restoration pass, which owns each chunk's visited
                                   words, then claims the binned heads exactly in LDS. 1 = on,
                                   -1 = off, 0 = library default (off: slower at R-MAT scale 24,
                                   where the scattered entry stores do not combine in L2). Bins
                                   are used only with sparse_frontier off (-1). */
} bfs_tunables;

/* ---- graph residency ------------------------------------------------------ */

/*
 * Make a CSR graph resident on the current HIP device. The graph is the
 * adjacency structure of section 3.3.1: row offsets and a column array of
 * neighbour ids (compressed sparse rows), which every later call reads.
 *   n        number of vertices, 1 <= n <= 2^31-1.
 *   nnz      number of arcs (directed CSR entries), 0 <= nnz <= 2^32 - 1.
 *   offsets  int64_t[n+1] (int32_t[n+1] with BFS_LOAD_OFFSETS_I32): row v is
 *            cols[offsets[v] .. offsets[v+1]). offsets[0]==0, offsets[n]==nnz,
 *            non-decreasing.
 *   cols     int32_t[nnz] out-neighbours, each in [0,n). Rows need not be sorted;
 *            self-loops and duplicate arcs are allowed and do not change levels.
 * The CSR is read as out-adjacency (any directed graph is accepted; a symmetric
 * CSR gives undirected BFS). Host inputs are copied and the library owns the
 * device copy; with BFS_LOAD_DEVICE_PTRS the caller's device arrays are used in
 * place. Returns BFS_E_INVALID_GRAPH when validation fails (nothing allocated).
 */
int bfs_graph_load_csr(int64_t n, int64_t nnz, const void* offsets, const int32_t* cols,
                       uint32_t flags, bfs_graph** out);

/* Release a graph and every buffer the library allocated for it.
 * BFS_E_BUSY if a server still holds it or a run on it is in progress on
 * another thread. NULL is accepted (no-op). */
int bfs_graph_free(bfs_graph* g);

/* Size of a resident graph; any output pointer may be NULL. device_bytes counts
 * library-owned device memory (CSR copy, hub table, cached workspaces). */
int bfs_graph_info(const bfs_graph* g, int64_t* n, int64_t* nnz, int64_t* device_bytes);

/* Read or replace the tunables used by later runs on this graph. Replacing them
 * may rebuild tables shared by every run on the graph (the big-row table, the
 * degree-ordered copy) and drops cached workspaces, so it returns BFS_E_BUSY
 * while a server holds the graph or a run on it is in progress on another
 * thread; it waits for asynchronous runs already enqueued (BFS_ASYNC) to finish
 * before rebuilding. BFS_E_INVALID_ARG for a combination that cannot run
 * (lds_visited on with a bitmap too large for LDS). */
int bfs_graph_get_tunables(const bfs_graph* g, bfs_tunables* t);
int bfs_graph_set_tunables(bfs_graph* g, const bfs_tunables* t);

/* ---- single-root BFS -------------------------------------------------------- */

/*
 * One top-down BFS from `root` (section 3.1, Algorithm 1; parallel form of
 * section 3.2, Algorithm 2, with the bitmap data structures of section 3.3.1).
 *   levels, parents  int32_t[n] each, written in full (caller-allocated; device
 *                    pointers unless BFS_OUT_HOST).
 *   stream           hipStream_t or NULL.
 *   flags            BFS_OUT_HOST, BFS_ASYNC (not both); BFS_HYBRID lets levels with large
 *                    frontiers run bottom-up (the direction-optimising hybrid the paper
 *                    names in its related work and conclusions: an unvisited vertex takes
 *                    the first frontier neighbour it finds as parent). arcs_scanned stays
 *                    the sum of degrees of the reached vertices.
 *   st               nullable; filled on return (must be NULL with BFS_ASYNC).
 * Errors: BFS_E_ROOT_RANGE, BFS_E_INVALID_ARG (also BFS_HYBRID on a graph not loaded
 * with BFS_LOAD_SYMMETRIC), BFS_E_DEVICE, BFS_E_NO_MEMORY. BFS_DETERMINISTIC works on
 * any graph: on a symmetric one each vertex scans its own row (stopping at the first
 * hit when rows are sorted), otherwise every reached vertex offers itself to its
 * out-neighbours with atomicMin.
 * Reentrant for distinct streams and outputs on the same graph.
 */
int bfs_run(bfs_graph* g, int32_t root, int32_t* levels, int32_t* parents, void* stream,
            uint32_t flags, bfs_run_stats* st);

/*
 * bfs_run without allocation, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same kernels and results as bfs_run (levels exact, parents
 * valid). Every scratch buffer of the run comes from one device array of
 * BFS_NOALLOC_SCRATCH_BYTES bytes that the library holds on each device it
 * runs on until the process ends; the caller passes only the graph, the root
 * and the outputs.
 *   levels, parents  device int32_t[n] each (host outputs would need staging).
 *   stream           hipStream_t or NULL; the call returns when the run is done.
 *   flags            0 or BFS_HYBRID (as for bfs_run).
 * Calls on one device share the array and are serialised inside the process
 * (each call completes before the next starts); the array keeps the last
 * call's contents, and the run clears what must start at zero. Runs on the
 * graph's current tunables and tables, and, like bfs_run, holds the graph
 * against bfs_graph_set_tunables for its duration.
 * Errors: BFS_E_NO_MEMORY when the run needs more scratch than the array
 * (bitmaps of 3n/8 bytes plus lists, and 8n bytes of run records when the
 * graph uses the degree-ordered copy): nothing is launched; BFS_E_ROOT_RANGE,
 * BFS_E_INVALID_ARG (NULL pointers, other flags, BFS_HYBRID on a graph not
 * loaded as symmetric), BFS_E_DEVICE. No hipMalloc, hipFree, host-pinned
 * allocation or event creation happens in this call.
 */
#define BFS_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int bfs_run_noalloc(bfs_graph* g, int32_t root, int32_t* levels, int32_t* parents, void* stream,
                    uint32_t flags);

/* ---- batched multi-source BFS --------------------------------------------------- */

/*
 * Independent BFS from each of num_roots roots, computed together: each root
 * follows the layer-by-layer procedure of section 3.1, Algorithm 1 (the
 * outputs are defined exactly as for bfs_run), and a group of up to 64 roots
 * shares one pass over each row, every vertex carrying a 64-bit visited /
 * frontier mask (bit i = root i of the group). Results are exactly those of
 * num_roots separate bfs_run calls (levels identical, parents valid).
 *   roots    host int32_t[num_roots]; duplicates allowed.
 *   levels   int32_t[num_roots * n], row-major: root i's levels at [i*n, (i+1)*n).
 *   parents  int32_t[num_roots * n], same layout.
 * Flags and stats as for bfs_run (stats are summed over roots).
 */
int bfs_run_batch(bfs_graph* g, const int32_t* roots, int32_t num_roots, int32_t* levels,
                  int32_t* parents, void* stream, uint32_t flags, bfs_run_stats* st);

/* ---- autotuner ------------------------------------------------------------- */

/*
 * Time candidate tunables on this graph with the given sample roots and keep
 * the fastest (also applied to the graph). mode 0 tunes bfs_run, mode 1 tunes
 * bfs_run_batch. Candidate results are checked against the default
 * configuration's levels; a candidate that differs is rejected. best may be NULL.
 * Changes the graph's tunables as bfs_graph_set_tunables does, with the same
 * BFS_E_BUSY rule (a graph held by a server cannot be tuned).
 */
int bfs_autotune(bfs_graph* g, const int32_t* roots, int32_t num_roots, int32_t mode,
                 bfs_tunables* best);

/* ---- serving --------------------------------------------------------------- */

typedef struct {
    int64_t mem_budget_bytes;       /* device bytes for instances and results; 0 = 50% of free */
    int32_t max_slots;              /* roots per multi-source instance (1..64); 0 = 64 */
    int32_t num_streams;            /* HIP streams shared by instances; 0 = 16 */
    int32_t max_instances_per_graph;/* concurrent instances of one graph; 0 = 3 */
    int32_t flags;                  /* reserved, must be 0 */
    int32_t single_workers;         /* reserved: must be 0 or -1 (every request is batched). A
                                       value above 0 asked for threads serving lightly loaded
                                       graphs with single-root runs; that route is disabled and
                                       bfs_server_create returns BFS_E_INVALID_ARG for it */
    int32_t batch_min_queue;        /* reserved for the single-root route (>= 0; ignored) */
} bfs_server_config;

typedef struct {
    int32_t num_levels;
    int32_t graph_id;
    int64_t reached;
    int64_t arcs_scanned;
    int64_t edges_traversed;
    double queue_ms;    /* submit -> admitted into an instance slot or to a worker */
    double latency_ms;  /* submit -> result complete on the device */
    int32_t batched;    /* 1 = served by a multi-source instance, 0 = by a single-root run */
    int32_t reserved;
} bfs_request_stats;

/* Start a server (a scheduler thread plus HIP streams). cfg may be NULL. */
int bfs_server_create(const bfs_server_config* cfg, bfs_server** out);

/* Register a resident graph; the server borrows it until destroyed. */
int bfs_server_add_graph(bfs_server* s, bfs_graph* g, int32_t* graph_id);

/* Queue one BFS request (thread-safe). A ticket is returned for polling. */
int bfs_server_submit(bfs_server* s, int32_t graph_id, int32_t root, uint64_t* ticket);

/*
 * Poll a ticket (thread-safe). BFS_PENDING while queued or running; BFS_OK once
 * done: levels/parents (int32_t[n] each; host or device pointers, copied with
 * hipMemcpyDefault; either may be NULL to skip) receive the result, st
 * (nullable) the request's stats, and the ticket is consumed.
 */
int bfs_server_poll(bfs_server* s, uint64_t ticket, int32_t* levels, int32_t* parents,
                    bfs_request_stats* st);

/* Stop the scheduler, drop pending requests and free server memory. */
int bfs_server_destroy(bfs_server* s);

/* Human-readable name of a status code (static string, never NULL). */
const char* bfs_status_str(int status);

#ifdef __cplusplus
}
#endif

#endif /* BFS_H */
