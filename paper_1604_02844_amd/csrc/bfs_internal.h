// Internal declarations of libbfs: graph residency, workspaces, launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/bfs.h"

namespace bfs {

// An error that maps to one ABI status code.
struct Error : std::runtime_error {
    int status;
    Error(int s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

[[noreturn]] void fail(int status, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define BFS_HIP(call) ::bfs::hip_check((call), #call)

constexpr int kStripes = 64;       // striped counters: one 128-byte line each
constexpr int kStripeStride = 16;  // u64 per stripe (128 bytes)

// Device-side control block of one run. Per-level counters are striped over
// separate cache lines (device-scope atomics on one address serialise) and
// double-buffered by level parity.
struct Ctrl {
    // Vertices found per level (slot 0 of each 128-byte stripe); with small
    // levels on, slot 1 sums the arcs of the rows restore blocks listed and
    // slot 2 the ids they listed (blocks that found too many list none).
    unsigned long long newcnt[2][kStripes * kStripeStride];
    unsigned long long bigarcs[2][kStripes * kStripeStride]; // arcs of the level's big rows
    unsigned long long reached;    // totals, written by the final stats kernel
    unsigned long long arcs;
    unsigned long long alive[3];   // multi-source: OR of new root bits per level (ring)
    unsigned long long newcnt_ms[3];
    int done;                      // set by the first level that finds an empty frontier
    int num_levels;
    int status;
    int steps;                     // single-root: expand/restore steps the run used (set when it ends)
    // Direction-optimising runs, indexed by level parity: the direction chosen
    // for the level (1 = bottom-up) and the vertices visited before its frontier.
    int dir[2];
    unsigned long long visited[2];
    // Levels a step's expansion ran beyond its own, indexed by step parity:
    // step s works on level s + shift[s & 1] and its expansion writes
    // shift[(s + 1) & 1] (so a late workgroup of step s still reads its own).
    int shift[2];
    // Whether the expansion of a level (indexed by its parity) put the heads of
    // its big-row arcs into destination bins for the restoration pass to claim.
    int binned[2];
};

// Scratch of one single-root run.
struct Workspace {
    int device = 0;
    int64_t words = 0;              // 32-bit words per bitmap (padded to 64)
    uint32_t* vis = nullptr;        // visited bits, updated during a level
    uint32_t* vis_prev = nullptr;   // exact visited bits at the start of the level
    uint32_t* fr = nullptr;         // exact frontier bits of the current level
    Ctrl* ctrl = nullptr;
    int last_launches = 0;          // level steps the previous single-root run needed
    // Next frontier of each restore block, listed when it is small: up to
    // kSmallSeg ids per block, and the block's count (above kSmallSeg: not all listed).
    int32_t* sl = nullptr;
    int32_t* sl_cnt = nullptr;
    unsigned long long* slots = nullptr;  // per-block partial sums (arcs | reached)
    int64_t nslots = 0;
    // Frontier rows above T2, compacted by the restore pass into one segment per
    // restore block: row ids, arc offsets within the segment, segment totals.
    int32_t* bl_u = nullptr;
    uint32_t* bl_pre = nullptr;
    uint32_t* seg_cnt = nullptr;
    uint32_t* seg_arcs = nullptr;
    int32_t big_capacity = 0;
    uint32_t* hot_vis = nullptr;    // compact visited bitmap of the hot vertices (ids 32r)
    uint32_t* hot_fr = nullptr;     // compact frontier bitmap of the hot vertices
    int32_t hot_capacity = 0;       // its words
    int32_t* run_rec = nullptr;     // {level, parent} per degree-ordered id (runs on the copy)
    // Destination bins of one level's big-row arcs: a bin per restore chunk
    // (256 visited words, 8192 vertices), a region of bin_k entries per
    // (bin, expansion workgroup); entries are {head, parent as a caller id}.
    int2* bin_e = nullptr;
    int64_t bin_cap = 0;            // entries
    uint32_t* bin_cnt = nullptr;    // [workgroup][bin] entries written
    int64_t bin_cnt_cap = 0;
    Ctrl* host_ctrl = nullptr;      // pinned mirror for stats
    int32_t* out_levels = nullptr;  // staging for BFS_OUT_HOST
    int32_t* out_parents = nullptr;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_free = nullptr;
    bool used = false;
    int64_t bytes = 0;
};

// Device control block of a multi-source instance (64 root slots).
struct MsCtrl {
    // Striped per-level statistics, double-buffered by level parity:
    // discoveries, arcs of the next frontier's rows, OR of discovered slot bits.
    unsigned long long disc[2][kStripes * kStripeStride];
    unsigned long long arcs[2][kStripes * kStripeStride];
    unsigned long long alive[2][kStripes * kStripeStride];
    unsigned long long work[kStripes * kStripeStride];  // batch: sum of deg(v) * roots holding v
    unsigned long long slot_reached[64];  // per-slot totals (serving)
    unsigned long long slot_arcs[64];
    int32_t* out_lv[64];                  // per-slot output rows
    int32_t* out_pa[64];
    int32_t start[64];                    // level at which each slot joined
    unsigned long long active;            // slots still running (host-managed)
    unsigned long long sum_disc;          // summary of one parity (k_ms_summary)
    unsigned long long sum_arcs;
    unsigned long long sum_alive;
    unsigned long long total_disc;        // batch totals
    unsigned long long total_arcs;
    int done;
    int num_levels;
};

// Scratch of one multi-source instance: masks, frontier double buffer, control.
struct MsWorkspace {
    int device = 0;
    int64_t n = 0;
    unsigned long long* vis = nullptr;
    unsigned long long* fr[2] = {nullptr, nullptr};
    MsCtrl* ctrl = nullptr;
    MsCtrl* host_ctrl = nullptr;  // pinned mirror
    int32_t* out_levels = nullptr;  // staging for BFS_OUT_HOST ([64*n])
    int32_t* out_parents = nullptr;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_free = nullptr;
    bool used = false;
    int64_t bytes = 0;
    int last_levels = 0;  // level steps the previous batch on this workspace enqueued until it ended (0: none yet)
    double last_unreached = 1.0;  // fraction of (root, vertex) pairs the previous batch left unreached
};

// Rows with degree above a threshold, for one vertex order: their ids, the
// exclusive prefix of their degrees, a bitmap that removes them from the
// per-wavefront frontier scan, and the capacity of each restore block's
// segment of the per-level big-row list.
struct BigTable {
    int32_t threshold = 0;
    int32_t num_big = 0;
    int64_t big_arcs = 0;
    int32_t* d_big = nullptr;
    int64_t* d_big_prefix = nullptr;
    uint32_t* d_bigmap = nullptr;
    int32_t* d_seg_start = nullptr;
    uint32_t* d_nzmap = nullptr;  // vertices with at least one arc (the only ones a bottom-up level can find)
    int64_t bytes = 0;
};

// Degree-ordered copy of the graph for single-root runs. The `hot` vertices of
// highest degree take ids 32r (r < hot): bit 0 of visited word r, so their
// visited bits form a compact bitmap that fits in LDS. Every other vertex keeps
// its relative order, so frontier words stay as evenly loaded as in the
// caller's order. Offsets are int64; outputs are written at caller ids.
// Hot vertices of the degree-ordered copy: degree rank s (0 = highest) sits
// at bit position (s / span) << shift of visited word s % span, so each of the
// first span = hot >> (5 - shift) words holds one hot vertex (shift 5) or two,
// at bits 0 and 16 (shift 4). The compact hot bitmaps use bit s.
inline int hot_shift_for(int64_t n, int64_t hot) { return hot <= n / 32 ? 5 : 4; }

struct HotLayout {
    int32_t hot = 0;
    int32_t shift = 5;  // hot_shift_for(n, hot)
    int32_t span = 0;   // visited words holding hot vertices
    int64_t* d_off = nullptr;       // [n+1], new order
    int32_t* d_col = nullptr;       // [nnz], new ids
    int32_t* d_new2old = nullptr;   // [n] run id -> caller id
    int32_t* d_old2new = nullptr;   // [n] caller id -> run id
    std::vector<int32_t> old2new;   // host copy, for the root
    BigTable big;
    // Destination blocks of the rows above T2 (all of them hot, so a row's
    // hot rank indexes its entry): block_vertices as requested (-1 = off);
    // when nblk > 0 those rows list their columns grouped by block
    // (id >> blk_shift, ascending) and bseg holds nblk + 1 local arc offsets
    // per row, the first arc of each block and the degree.
    int32_t blk_req = -1;
    int32_t blk_shift = 0;
    int32_t nblk = 0;
    uint32_t* d_bseg = nullptr;
    int64_t bytes = 0;
};

}  // namespace bfs

struct bfs_graph {
    int device = 0;
    int64_t n = 0, nnz = 0;
    bool off32 = false;        // 4-byte offsets on the device
    bool owns = true;          // device arrays allocated by the library
    bool symmetric = false;    // loaded with BFS_LOAD_SYMMETRIC (checked unless validation is skipped)
    bool rows_sorted = false;  // symmetric graphs: every row lists ids in non-decreasing order
    void* d_off = nullptr;     // int64_t[n+1] or int32_t[n+1]
    int32_t* d_col = nullptr;  // int32_t[nnz]
    int64_t max_degree = 0;
    int cu_count = 0;

    // Rows above T2 in the caller's order (split over the whole grid).
    bfs::BigTable big;
    // Restore grid (one big-row list segment per restore block).
    int32_t restore_grid = 0;
    // Degree-ordered copy for single-root runs with an LDS hot bitmap.
    std::unique_ptr<bfs::HotLayout> hot;

    bfs_tunables tun{};     // guarded by mu
    std::mutex mu;
    int ws_out = 0;         // workspaces checked out (single-root and multi-source), guarded by mu
    std::vector<bfs::Workspace*> ws_free;
    std::vector<bfs::Workspace*> ws_all;
    std::vector<bfs::MsWorkspace*> ms_free;
    std::vector<bfs::MsWorkspace*> ms_all;
    std::atomic<int> server_refs{0};
    int64_t device_bytes = 0;
};

namespace bfs {

bfs_tunables default_tunables(const bfs_graph* g);
bfs_tunables resolve_tunables(const bfs_graph* g, const bfs_tunables& t);
// Make the graph's derived tables match resolved tunables `r` (big-row tables
// of both orders, the degree-ordered copy) and store them. BFS_E_BUSY while a
// server holds the graph or any workspace is checked out (a run in progress on
// another thread, a server instance): rebuilding would free memory those use.
// Waits for in-flight asynchronous work first when anything has to be rebuilt.
// Caller must not hold g->mu.
void apply_tunables(bfs_graph* g, const bfs_tunables& r);
void build_big_table(bfs::BigTable& t, const void* d_off, bool off32, int64_t n, int32_t threshold, int restore_grid,
                     int cu_count, int64_t* max_degree);
void free_big_table(bfs::BigTable& t);
// Hot vertices used for these tunables (0 = no degree-ordered copy).
int32_t hot_count(const bfs_graph* g, const bfs_tunables& t);
// `blk`: resolved block_vertices tunable (-1 = no destination blocks).
void build_hot_layout(bfs_graph* g, int32_t hot, int32_t threshold, int32_t blk);
// Most destination blocks a grouped row may span (one per lane of a wavefront).
constexpr int kMaxBlocks = 64;
void free_hot_layout(bfs_graph* g);
// Device part of the copy (single.hip): new columns of every new row.
// Rows above big_threshold are grouped by destination block when nblk > 0
// (offsets into bseg by hot rank).
void launch_relabel_cols(const bfs_graph* g, const int64_t* d_noff, const int32_t* d_new2old,
                         const int32_t* d_old2new, int32_t* d_ncol, int32_t hot_span, int32_t hot_shift,
                         int32_t big_threshold, int32_t blk_shift, int32_t nblk, uint32_t* d_bseg);
int64_t padded_words(int64_t n);
// Most visited-bitmap words an expansion workgroup of `block` threads can hold
// in LDS beside its static shared memory.
int64_t lds_visited_words_max(int block);
// Visited-bitmap words a single-root run keeps in LDS (0 = none).
int64_t lds_visited_words(const bfs_graph* g, const bfs_tunables& t);
// Blocks of the restore pass: 256-word chunks, chunk c handled by block c % grid.
constexpr int kRestoreBlock = 256;
// Upper bound of the restore grid (= number of big-row list segments); the
// expansion kernel keeps two prefix arrays of this length in LDS.
constexpr int kMaxRestoreGrid = 1024;
// Largest LDS snapshot of hot visited words per expansion workgroup (128 KiB).
constexpr int kMaxHotWords = 32768;
constexpr int kSmallSeg = 64;      // listed next-frontier ids per restore block
constexpr int kSmallMax = 4096;    // largest frontier one expansion workgroup takes alone
int restore_grid_for(int64_t words, int cu_count);

// Workspaces are checked out under g->mu; `t` (nullable) receives the graph's
// resolved tunables read under the same lock, so a run's tunables and the
// derived tables they select cannot change while it holds the workspace
// (apply_tunables refuses with BFS_E_BUSY while any workspace is out).
Workspace* acquire_ws(bfs_graph* g, hipStream_t s, bfs_tunables* t = nullptr);
void release_ws(bfs_graph* g, Workspace* w, hipStream_t s);
// Bytes one single-root workspace of this graph needs (for its current tables;
// with `bins`, also the destination bins of hub levels). With `base` (256-byte
// aligned, that many bytes) the workspace's buffers are also carved from it;
// events and the host mirror are left to the caller.
size_t ws_layout(const bfs_graph* g, Workspace* w, char* base, bool bins = true);
// Most expansion workgroups whose bins a workspace holds counts for.
constexpr int kMaxBinGroups = 2048;
MsWorkspace* acquire_ms(bfs_graph* g, hipStream_t s, bfs_tunables* t = nullptr);
void release_ms(bfs_graph* g, MsWorkspace* w, hipStream_t s);
// The graph's resolved tunables, read under g->mu.
bfs_tunables current_tunables(bfs_graph* g);
void free_workspaces(bfs_graph* g);

// Launchers (the kernels live in single.hip and multi.hip).
// stop (nullable) is recorded on s right after the run's last kernel, before
// the host learns that the run has ended.
void launch_single(bfs_graph* g, const bfs_tunables& t, Workspace* w, int32_t root, int32_t* levels,
                   int32_t* parents, hipStream_t s, bool hybrid = false, hipEvent_t stop = nullptr);
void launch_single_stats(Workspace* w, hipStream_t s);
// Stats of a run from its level array (hybrid runs scan no frontier rows in
// bottom-up levels): reached and the sum of their degrees.
void launch_single_stats_from_levels(bfs_graph* g, const bfs_tunables& t, Workspace* w, const int32_t* levels,
                                     hipStream_t s);
// Symmetry check of a resident CSR (a multiset hash of arcs against reversed arcs).
bool csr_is_symmetric(const bfs_graph* g);
bool csr_rows_sorted(const bfs_graph* g);
// Deterministic predecessors (BFS_DETERMINISTIC): after a run, parents[v] = the
// least in-neighbour one level up, on the caller's ids (parents.hip).
void launch_least_parents(const bfs_graph* g, const int32_t* levels, int32_t* parents, hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t s);

// Multi-source engine (multi.hip). A batch runs every level device-side with
// chunked host checks; the server steps one level at a time.
void ms_run_batch(bfs_graph* g, const bfs_tunables& t, MsWorkspace* w, const int32_t* roots, int32_t count,
                  int32_t* levels, int32_t* parents, int64_t ld, hipStream_t s, hipEvent_t stop = nullptr);
void ms_reset(bfs_graph* g, MsWorkspace* w, hipStream_t s);
// Seed slots (host arrays) into the frontier of instance level `level`: root
// bits and level-0 outputs. The slot output pointers and start levels must
// already be in w->ctrl. With `pinned_stage` (128 int32 of pinned host memory,
// untouched until `s` has passed this point) nothing blocks; without it the
// call waits for the stream.
void ms_join(bfs_graph* g, MsWorkspace* w, const int32_t* slots, const int32_t* roots, int32_t count, int level,
             hipStream_t s, int32_t* pinned_stage);
// Enqueue one level of the instance on `s` plus an asynchronous copy of the
// step summary (sum_*, per-slot totals) into w->host_ctrl; the caller
// synchronises `s` before reading it. `level` is the instance level expanded.
void ms_step_enqueue(bfs_graph* g, const bfs_tunables& t, MsWorkspace* w, int level, hipStream_t s,
                     bool per_slot);
// Point slot `slot` at its output rows and start level (host-side staging in
// `staging`, a pinned MsCtrl that must stay untouched until `s` has drained).
void ms_set_slot(MsWorkspace* w, MsCtrl* staging, int slot, int32_t* lv, int32_t* pa, int32_t start,
                 hipStream_t s);
void ms_retire(bfs_graph* g, MsWorkspace* w, unsigned long long keep, hipStream_t s);

int device_cu_count(int device);

}  // namespace bfs
