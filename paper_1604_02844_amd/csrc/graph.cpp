// Graph residency: CSR validation and upload, the big-row table, tunables and
// workspace pools.
#include <algorithm>
#include <cstring>

#include "bfs_internal.h"

namespace bfs {

void fail(int status, const std::string& msg) { throw Error(status, msg); }

void hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        fail(BFS_E_NO_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
    }
    fail(BFS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int device_cu_count(int device) {
    int cus = 0;
    BFS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    return cus;
}

namespace {

template <typename OffT>
void validate_host(int64_t n, int64_t nnz, const OffT* off, const int32_t* col) {
    if (off[0] != 0) fail(BFS_E_INVALID_GRAPH, "offsets[0] != 0");
    for (int64_t v = 0; v < n; ++v)
        if (off[v + 1] < off[v]) fail(BFS_E_INVALID_GRAPH, "offsets decrease at row " + std::to_string(v));
    if ((int64_t)off[n] != nnz) fail(BFS_E_INVALID_GRAPH, "offsets[n] != nnz");
    for (int64_t j = 0; j < nnz; ++j)
        if (col[j] < 0 || col[j] >= n) fail(BFS_E_INVALID_GRAPH, "column out of range at arc " + std::to_string(j));
}

template <typename OffT>
std::vector<int64_t> degrees_of(int64_t n, const OffT* off) {
    std::vector<int64_t> d((size_t)n);
    for (int64_t v = 0; v < n; ++v) d[(size_t)v] = (int64_t)off[v + 1] - (int64_t)off[v];
    return d;
}

}  // namespace

// Device-side CSR checks for borrowed device arrays (kernel in single.hip).
void validate_device_csr(const void* off, bool off32, const int32_t* col, int64_t n, int64_t nnz);

int64_t padded_words(int64_t n) {
    int64_t words = (n + 31) / 32;
    return (words + 63) / 64 * 64;
}

int restore_grid_for(int64_t words, int cu_count) {
    const int64_t chunks = (words + kRestoreBlock - 1) / kRestoreBlock;
    const int64_t cap = std::min<int64_t>((int64_t)std::max(cu_count, 1) * 4, kMaxRestoreGrid);
    return (int)std::max<int64_t>(1, std::min<int64_t>(chunks, cap));
}

namespace {

std::vector<int64_t> host_offsets(const void* d_off, bool off32, int64_t n) {
    std::vector<int64_t> off((size_t)n + 1);
    if (off32) {
        std::vector<int32_t> o32((size_t)n + 1);
        BFS_HIP(hipMemcpy(o32.data(), d_off, o32.size() * 4, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < o32.size(); ++i) off[i] = o32[i];
    } else {
        BFS_HIP(hipMemcpy(off.data(), d_off, off.size() * 8, hipMemcpyDeviceToHost));
    }
    return off;
}

}  // namespace

void free_big_table(BigTable& t) {
    if (t.d_big) (void)hipFree(t.d_big);
    if (t.d_big_prefix) (void)hipFree(t.d_big_prefix);
    if (t.d_bigmap) (void)hipFree(t.d_bigmap);
    if (t.d_seg_start) (void)hipFree(t.d_seg_start);
    if (t.d_nzmap) (void)hipFree(t.d_nzmap);
    t = BigTable{};
}

// Rows with degree > threshold (split over the whole expansion grid) and the
// bitmap that removes them from the per-wavefront frontier scan.
void build_big_table(BigTable& t, const void* d_off, bool off32, int64_t n, int32_t threshold, int restore_grid,
                     int cu_count, int64_t* max_degree) {
    (void)cu_count;
    if (threshold < 1) threshold = 1;
    free_big_table(t);
    t.threshold = threshold;
    const std::vector<int64_t> off = host_offsets(d_off, off32, n);
    const int64_t words = padded_words(n);
    std::vector<uint32_t> bigmap((size_t)words, 0u), nzmap((size_t)words, 0u);
    std::vector<int32_t> big;
    std::vector<int64_t> prefix(1, 0);
    int64_t maxd = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t d = off[(size_t)v + 1] - off[(size_t)v];
        maxd = std::max(maxd, d);
        if (d > 0) nzmap[(size_t)(v >> 5)] |= 1u << (v & 31);
        if (d > threshold) {
            big.push_back((int32_t)v);
            prefix.push_back(prefix.back() + d);
            bigmap[(size_t)(v >> 5)] |= 1u << (v & 31);
        }
    }
    if (max_degree) *max_degree = maxd;
    t.num_big = (int32_t)big.size();
    t.big_arcs = prefix.back();
    try {
        BFS_HIP(hipMalloc(&t.d_big, std::max<size_t>(big.size(), 1) * 4));
        BFS_HIP(hipMalloc(&t.d_big_prefix, prefix.size() * 8));
        BFS_HIP(hipMalloc(&t.d_bigmap, (size_t)words * 4));
        if (!big.empty()) BFS_HIP(hipMemcpy(t.d_big, big.data(), big.size() * 4, hipMemcpyHostToDevice));
        BFS_HIP(hipMemcpy(t.d_big_prefix, prefix.data(), prefix.size() * 8, hipMemcpyHostToDevice));
        BFS_HIP(hipMemcpy(t.d_bigmap, bigmap.data(), (size_t)words * 4, hipMemcpyHostToDevice));
        BFS_HIP(hipMalloc(&t.d_nzmap, (size_t)words * 4));
        BFS_HIP(hipMemcpy(t.d_nzmap, nzmap.data(), (size_t)words * 4, hipMemcpyHostToDevice));
        // Segment capacities of the restore pass: the big rows inside the
        // chunks that each restore block visits.
        std::vector<int32_t> seg((size_t)restore_grid + 1, 0);
        for (int64_t w = 0; w < words; ++w) {
            const int b = (int)((w / kRestoreBlock) % restore_grid);
            seg[(size_t)b + 1] += __builtin_popcount(bigmap[(size_t)w]);
        }
        for (int b = 0; b < restore_grid; ++b) seg[(size_t)b + 1] += seg[(size_t)b];
        BFS_HIP(hipMalloc(&t.d_seg_start, seg.size() * 4));
        BFS_HIP(hipMemcpy(t.d_seg_start, seg.data(), seg.size() * 4, hipMemcpyHostToDevice));
        t.bytes = (int64_t)std::max<size_t>(big.size(), 1) * 4 + (int64_t)prefix.size() * 8 + words * 8 +
                  (int64_t)seg.size() * 4;
    } catch (...) {
        free_big_table(t);
        throw;
    }
}

int32_t hot_count(const bfs_graph* g, const bfs_tunables& t) {
    if (t.hot_vertices <= 0) return 0;
    // Whole 64-bit words of the compact bitmap, at most two per full visited word.
    int64_t h = ((int64_t)t.hot_vertices + 63) / 64 * 64;
    h = std::min<int64_t>(h, (int64_t)kMaxHotWords * 32);
    h = std::min<int64_t>(h, g->n / 32 * 2 / 64 * 64);
    return (int32_t)std::max<int64_t>(h, 0);
}

void free_hot_layout(bfs_graph* g) {
    if (!g->hot) return;
    HotLayout& h = *g->hot;
    if (h.d_off) (void)hipFree(h.d_off);
    if (h.d_col) (void)hipFree(h.d_col);
    if (h.d_new2old) (void)hipFree(h.d_new2old);
    if (h.d_old2new) (void)hipFree(h.d_old2new);
    if (h.d_bseg) (void)hipFree(h.d_bseg);
    free_big_table(h.big);
    g->device_bytes -= h.bytes;
    g->hot.reset();
}

// The degree-ordered copy. Hot vertices: the `hot` highest degrees (ties to
// the lower id), by decreasing degree at bit 0 of the first `span` visited
// words, then (when they need two per word) at bit 16 of the same words; all
// other vertices fill the remaining ids in increasing caller-id order. Columns are renamed on
// the device and every row lists its hot neighbours first (each part in the
// original arc order), so a bottom-up scan meets the likely parents first.
void build_hot_layout(bfs_graph* g, int32_t hot, int32_t threshold, int32_t blk) {
    free_hot_layout(g);
    if (hot <= 0) return;
    const int64_t n = g->n;
    const std::vector<int64_t> off = host_offsets(g->d_off, g->off32, n);
    // Degree threshold D with #(deg > D) < hot <= #(deg >= D), by a histogram.
    int64_t maxd = 0;
    for (int64_t v = 0; v < n; ++v) maxd = std::max(maxd, off[(size_t)v + 1] - off[(size_t)v]);
    std::vector<int64_t> cnt((size_t)maxd + 2, 0);
    for (int64_t v = 0; v < n; ++v) ++cnt[(size_t)(off[(size_t)v + 1] - off[(size_t)v])];
    int64_t D = maxd, above = 0;
    while (D > 0 && above + cnt[(size_t)D] < hot) above += cnt[(size_t)D--];
    int64_t take_eq = hot - above;  // vertices of degree exactly D still needed
    std::vector<char> is_hot((size_t)n, 0);
    std::vector<int32_t> hot_ids;
    hot_ids.reserve((size_t)hot);
    for (int64_t v = 0; v < n && (int64_t)hot_ids.size() < hot; ++v) {
        const int64_t d = off[(size_t)v + 1] - off[(size_t)v];
        if (d > D || (d == D && take_eq > 0)) {
            if (d == D) --take_eq;
            is_hot[(size_t)v] = 1;
            hot_ids.push_back((int32_t)v);
        }
    }
    if ((int64_t)hot_ids.size() != hot) fail(BFS_E_INTERNAL, "hot vertex selection");
    // Hot rank r goes to the r-th highest degree (ties to the lower id).
    std::stable_sort(hot_ids.begin(), hot_ids.end(), [&](int32_t a, int32_t b) {
        return off[(size_t)a + 1] - off[(size_t)a] > off[(size_t)b + 1] - off[(size_t)b];
    });
    const int shift = hot_shift_for(n, hot);
    const int64_t span = (int64_t)(hot / 32) << shift;
    if (hot % 64 != 0 || span * 32 > n) fail(BFS_E_INTERNAL, "hot set does not fit the visited words");
    std::vector<int32_t> new2old((size_t)n), old2new((size_t)n);
    int64_t cold = 0;
    for (int64_t x = 0; x < n; ++x) {
        // Position k = (x & 31) >> shift of word x >> 5 holds rank (x >> 5) + k * span.
        if ((x & ((1 << shift) - 1)) == 0 && (x >> 5) < span) {
            new2old[(size_t)x] = hot_ids[(size_t)((x >> 5) + ((x & 31) >> shift) * span)];
        } else {
            while (is_hot[(size_t)cold]) ++cold;
            new2old[(size_t)x] = (int32_t)cold++;
        }
        old2new[(size_t)new2old[(size_t)x]] = (int32_t)x;
    }
    std::vector<int64_t> noff((size_t)n + 1, 0);
    for (int64_t x = 0; x < n; ++x) {
        const int64_t u = new2old[(size_t)x];
        noff[(size_t)x + 1] = noff[(size_t)x] + (off[(size_t)u + 1] - off[(size_t)u]);
    }
    auto h = std::make_unique<HotLayout>();
    h->hot = hot;
    h->shift = shift;
    h->span = (int32_t)span;
    // Destination blocks for the rows above T2: only when every such row is
    // hot (its hot rank indexes the offsets) and a row spans at most
    // kMaxBlocks blocks.
    int64_t num_big = 0;
    for (int64_t v = 0; v < n; ++v) num_big += (off[(size_t)v + 1] - off[(size_t)v]) > threshold ? 1 : 0;
    h->blk_req = blk;
    if (blk > 0 && num_big > 0 && num_big <= hot) {
        int bs = 0;
        while (((int64_t)1 << bs) < blk) ++bs;
        const int64_t nb = (n + ((int64_t)1 << bs) - 1) >> bs;
        if (nb <= kMaxBlocks) {
            h->blk_shift = bs;
            h->nblk = (int32_t)nb;
        }
    }
    const size_t bseg_bytes = h->nblk > 0 ? (size_t)num_big * (size_t)(h->nblk + 1) * 4 : 0;
    try {
        BFS_HIP(hipMalloc(&h->d_off, noff.size() * 8));
        BFS_HIP(hipMalloc(&h->d_col, std::max<size_t>((size_t)g->nnz * 4, 4)));
        BFS_HIP(hipMalloc(&h->d_new2old, (size_t)n * 4));
        BFS_HIP(hipMalloc(&h->d_old2new, (size_t)n * 4));
        if (bseg_bytes) BFS_HIP(hipMalloc(&h->d_bseg, bseg_bytes));
        BFS_HIP(hipMemcpy(h->d_off, noff.data(), noff.size() * 8, hipMemcpyHostToDevice));
        BFS_HIP(hipMemcpy(h->d_new2old, new2old.data(), (size_t)n * 4, hipMemcpyHostToDevice));
        BFS_HIP(hipMemcpy(h->d_old2new, old2new.data(), (size_t)n * 4, hipMemcpyHostToDevice));
        launch_relabel_cols(g, h->d_off, h->d_new2old, h->d_old2new, h->d_col, h->span, h->shift, threshold,
                            h->blk_shift, h->nblk, h->d_bseg);
        BFS_HIP(hipDeviceSynchronize());
        build_big_table(h->big, h->d_off, false, n, threshold, g->restore_grid, g->cu_count, nullptr);
        if (h->big.num_big != g->big.num_big) fail(BFS_E_INTERNAL, "degree-ordered copy changed the big rows");
    } catch (...) {
        if (h->d_off) (void)hipFree(h->d_off);
        if (h->d_col) (void)hipFree(h->d_col);
        if (h->d_new2old) (void)hipFree(h->d_new2old);
        if (h->d_old2new) (void)hipFree(h->d_old2new);
        if (h->d_bseg) (void)hipFree(h->d_bseg);
        free_big_table(h->big);
        throw;
    }
    h->old2new = std::move(old2new);
    h->bytes = (int64_t)noff.size() * 8 + g->nnz * 4 + n * 8 + h->big.bytes + (int64_t)bseg_bytes;
    g->device_bytes += h->bytes;
    g->hot = std::move(h);
}

int64_t lds_visited_words(const bfs_graph* g, const bfs_tunables& t) {
    if (t.lds_visited <= 0 || hot_count(g, t) > 0) return 0;
    const int64_t words = padded_words(g->n);
    return words <= lds_visited_words_max(t.block_size) ? words : 0;
}

void apply_tunables(bfs_graph* g, const bfs_tunables& r) {
    if (r.lds_visited > 0 && hot_count(g, r) == 0 && padded_words(g->n) > lds_visited_words_max(r.block_size))
        fail(BFS_E_INVALID_ARG, "the visited bitmap does not fit in LDS beside this workgroup size");
    // Held for the whole call: a run that starts meanwhile waits in acquire_ws
    // and then sees the new tunables and tables together.
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->server_refs.load() > 0) fail(BFS_E_BUSY, "graph is registered with a server");
    if (g->ws_out > 0) fail(BFS_E_BUSY, "a run on this graph is in progress");
    const int32_t want_hot = hot_count(g, r);
    const bool big_stale = r.wave_max_degree != g->big.threshold;
    // The copy is rebuilt whole when its hot set or destination blocks change,
    // and when T2 changes while its rows above T2 are grouped by block (they
    // are grouped at build time); otherwise a new T2 only rebuilds its big-row table.
    const bool copy_stale = want_hot != (g->hot ? g->hot->hot : 0) ||
                            (g->hot && (g->hot->blk_req != r.block_vertices ||
                                        (g->hot->blk_req > 0 && g->hot->big.threshold != r.wave_max_degree)));
    const bool hot_stale = copy_stale || (g->hot && g->hot->big.threshold != r.wave_max_degree);
    if (r.hub_bins != resolve_tunables(g, g->tun).hub_bins && !big_stale && !hot_stale) {
        // Workspaces hold the bins only while they are on: drop them.
        BFS_HIP(hipDeviceSynchronize());
        for (auto* w : g->ws_all) g->device_bytes -= w->bytes;
        for (auto* w : g->ms_all) g->device_bytes -= w->bytes;
        free_workspaces(g);
    }
    if (big_stale || hot_stale) {
        // Tables are shared by every run on the graph: rebuild them only after
        // in-flight asynchronous work has drained. Workspaces hold lists sized
        // for the old tables: drop them (none is checked out).
        BFS_HIP(hipDeviceSynchronize());
        for (auto* w : g->ws_all) g->device_bytes -= w->bytes;
        for (auto* w : g->ms_all) g->device_bytes -= w->bytes;
        free_workspaces(g);
        if (big_stale) {
            g->device_bytes -= g->big.bytes;
            build_big_table(g->big, g->d_off, g->off32, g->n, r.wave_max_degree, g->restore_grid, g->cu_count,
                            &g->max_degree);
            g->device_bytes += g->big.bytes;
        }
        if (copy_stale) {
            build_hot_layout(g, want_hot, r.wave_max_degree, r.block_vertices);
        } else if (g->hot && g->hot->big.threshold != r.wave_max_degree) {
            HotLayout& h = *g->hot;
            g->device_bytes -= h.big.bytes;
            h.bytes -= h.big.bytes;
            build_big_table(h.big, h.d_off, false, g->n, r.wave_max_degree, g->restore_grid, g->cu_count, nullptr);
            g->device_bytes += h.big.bytes;
            h.bytes += h.big.bytes;
        }
    }
    g->tun = r;
}

bfs_tunables current_tunables(bfs_graph* g) {
    std::lock_guard<std::mutex> lk(g->mu);
    return resolve_tunables(g, g->tun);
}

bfs_tunables default_tunables(const bfs_graph* g) {
    bfs_tunables t{};
    (void)g;
    t.small_max_degree = 256;
    t.wave_max_degree = 256;
    t.chunk_arcs = 0;
    t.block_size = 256;
    t.blocks_per_cu = 0;  // 0 = as many as fit (occupancy query at launch)
    t.batch_width = 64;
    t.update_mode = 1;
    // From 2^22 vertices on, single-root runs use the degree-ordered copy with
    // an LDS bitmap of the 2^20 highest-degree vertices (128 KiB; fewer below
    // 2^25 vertices, at most two per visited word), shared by the 16
    // wavefronts of a 1024-thread workgroup.
    // Only skewed degree distributions concentrate probes on few vertices.
    const bool large = g && g->n >= (int64_t)1 << 22 &&
                       g->max_degree > 64 * std::max<int64_t>(1, g->nnz / std::max<int64_t>(1, g->n));
    t.hot_vertices = large ? 1 << 20 : -1;
    if (large) t.block_size = 1024;
    // Up to 2^20 vertices the whole visited bitmap (128 KiB) fits in the LDS
    // of a 1024-thread workgroup instead.
    const bool fits = g && !large && g->n >= (int64_t)1 << 16 &&
                      padded_words(g->n) <= lds_visited_words_max(1024);
    t.lds_visited = fits ? 1 : -1;
    t.sparse_frontier = 1024;  // the tail of small levels in one workgroup: R-MAT 20 -1%, 24/26 even
    // Destination-blocked expansion of the rows above T2: measured slower at
    // R-MAT scale 24 (the rows' arcs split into short per-block runs), so off.
    t.block_vertices = -1;
    // One cooperative launch per batch is measured slower than per-level
    // launches (R-MAT 22, 64 roots: 11.45 ms against 10.16 ms), so off.
    t.persistent = -1;
    // Hub-level destination bins: exact, but slower at R-MAT scale 24 (the
    // scattered entry stores do not combine in L2), so off.
    t.hub_bins = -1;
    if (fits) t.block_size = 1024;
    return t;
}

bfs_tunables resolve_tunables(const bfs_graph* g, const bfs_tunables& in) {
    bfs_tunables d = default_tunables(g), t = in;
    if (t.small_max_degree <= 0) t.small_max_degree = d.small_max_degree;
    // Packed rows are summed in 32-bit lanes of a wavefront scan: keep 64*T1 small.
    if (t.small_max_degree > 65536) t.small_max_degree = 65536;
    if (t.wave_max_degree <= 0) t.wave_max_degree = d.wave_max_degree;
    if (t.wave_max_degree < t.small_max_degree) t.wave_max_degree = t.small_max_degree;
    if (t.chunk_arcs < 0) t.chunk_arcs = 0;
    if (t.block_size != 256 && t.block_size != 512 && t.block_size != 1024) t.block_size = d.block_size;
    if (t.blocks_per_cu < 0) t.blocks_per_cu = 0;
    if (t.batch_width <= 0 || t.batch_width > 64) t.batch_width = d.batch_width;
    if (t.update_mode != 1 && t.update_mode != 2) t.update_mode = d.update_mode;
    // By default the LDS copy of the visited bitmap goes with 1024-thread
    // workgroups only: with fewer waves per copy it costs occupancy.
    if (t.lds_visited == 0) t.lds_visited = d.lds_visited > 0 && t.block_size == 1024 ? 1 : -1;
    t.lds_visited = t.lds_visited > 0 ? 1 : -1;
    if (t.sparse_frontier == 0) t.sparse_frontier = d.sparse_frontier;
    if (t.sparse_frontier < 0) t.sparse_frontier = -1;
    if (t.sparse_frontier > kSmallMax) t.sparse_frontier = kSmallMax;
    if (t.hot_vertices == 0) t.hot_vertices = d.hot_vertices;
    if (t.hot_vertices < 0) t.hot_vertices = -1;
    if (t.hot_vertices > kMaxHotWords * 32) t.hot_vertices = kMaxHotWords * 32;
    if (t.hub_bins == 0) t.hub_bins = d.hub_bins;
    t.hub_bins = t.hub_bins > 0 ? 1 : -1;
    if (t.persistent == 0) t.persistent = d.persistent;
    t.persistent = t.persistent > 0 ? 1 : -1;
    if (t.block_vertices == 0) t.block_vertices = d.block_vertices;
    if (t.block_vertices < 0) {
        t.block_vertices = -1;
    } else {
        int s = 11;
        while (s < 20 && ((int64_t)1 << (s + 1)) <= t.block_vertices) ++s;
        t.block_vertices = 1 << s;
    }
    return t;
}

// ---------------------------------------------------------------------------
// Workspace pools. A workspace returned to the pool records an event on the
// stream that used it; the next user on another stream waits for that event.
// ---------------------------------------------------------------------------

size_t ws_layout(const bfs_graph* g, Workspace* w, char* base, bool bins) {
    w->device = g->device;
    w->words = padded_words(g->n);
    w->nslots = (int64_t)g->cu_count * 64 + 64;  // >= any expansion or restore grid
    w->big_capacity = std::max(g->big.num_big, 1);
    const size_t bmb = (size_t)w->words * 4;
    const size_t listb = (size_t)w->big_capacity * 8 + (size_t)(g->restore_grid + 1) * 8;
    w->hot_capacity = (int)std::min<int64_t>(w->words / 16, kMaxHotWords);
    const size_t hotb = (size_t)w->hot_capacity * 8;  // visited and frontier bits
    const size_t recb = g->hot ? (size_t)g->n * 8 : 0;  // {level, parent} in the degree-ordered ids
    const size_t smallb = (size_t)g->restore_grid * (kSmallSeg + 1) * 4;  // listed small frontiers
    const size_t pre_rec = bmb * 3 + sizeof(Ctrl) + (size_t)w->nslots * 2 * 8 + listb + hotb + smallb;
    const size_t rec_at = (pre_rec + 255) & ~(size_t)255;
    // Destination bins: 4 entries per vertex (at least 2^16, at most 2^28) and
    // one count per (bin, workgroup) for up to kMaxBinGroups workgroups.
    const int64_t nbins = (w->words + kRestoreBlock - 1) / kRestoreBlock;
    bins = bins && resolve_tunables(g, g->tun).hub_bins > 0;  // only graphs that use them pay for them
    w->bin_cap = bins ? std::min<int64_t>(std::max<int64_t>(4 * g->n, (int64_t)1 << 16), (int64_t)1 << 28) : 0;
    w->bin_cnt_cap = bins ? nbins * kMaxBinGroups : 0;
    const size_t bin_at = (rec_at + recb + 255) & ~(size_t)255;
    const size_t cnt_at = bin_at + (size_t)w->bin_cap * 8;
    const size_t total = cnt_at + (size_t)w->bin_cnt_cap * 4;
    if (!base) return total;
    w->bin_e = bins ? reinterpret_cast<int2*>(base + bin_at) : nullptr;
    w->bin_cnt = bins ? reinterpret_cast<uint32_t*>(base + cnt_at) : nullptr;
    w->vis = reinterpret_cast<uint32_t*>(base);
    w->vis_prev = w->vis + w->words;
    w->fr = w->vis_prev + w->words;
    w->ctrl = reinterpret_cast<Ctrl*>(base + bmb * 3);
    w->slots = reinterpret_cast<unsigned long long*>(base + bmb * 3 + sizeof(Ctrl));
    char* lp = base + bmb * 3 + sizeof(Ctrl) + (size_t)w->nslots * 2 * 8;
    w->bl_u = reinterpret_cast<int32_t*>(lp);
    w->bl_pre = reinterpret_cast<uint32_t*>(lp + (size_t)w->big_capacity * 4);
    w->seg_cnt = reinterpret_cast<uint32_t*>(lp + (size_t)w->big_capacity * 8);
    w->seg_arcs = w->seg_cnt + (g->restore_grid + 1);
    w->hot_vis = reinterpret_cast<uint32_t*>(lp + listb);
    w->hot_fr = w->hot_vis + w->hot_capacity;
    w->run_rec = recb ? reinterpret_cast<int32_t*>(base + rec_at) : nullptr;
    w->sl = reinterpret_cast<int32_t*>(lp + listb + hotb);
    w->sl_cnt = w->sl + (size_t)g->restore_grid * kSmallSeg;
    w->bytes = (int64_t)total;
    return total;
}

Workspace* acquire_ws(bfs_graph* g, hipStream_t s, bfs_tunables* t) {
    std::lock_guard<std::mutex> lk(g->mu);
    Workspace* w = nullptr;
    if (!g->ws_free.empty()) {
        w = g->ws_free.back();
        g->ws_free.pop_back();
        if (w->used) {
            const hipError_t e = hipStreamWaitEvent(s, w->ev_free, 0);
            if (e != hipSuccess) {
                g->ws_free.push_back(w);
                hip_check(e, "hipStreamWaitEvent");
            }
        }
        if (t) *t = resolve_tunables(g, g->tun);
        ++g->ws_out;
        return w;
    }
    w = new Workspace();
    try {
        const size_t total = ws_layout(g, w, nullptr);
        char* base = nullptr;
        BFS_HIP(hipMalloc(&base, total));
        ws_layout(g, w, base);
        BFS_HIP(hipMemset(w->ctrl, 0, sizeof(Ctrl)));
        BFS_HIP(hipHostMalloc(&w->host_ctrl, sizeof(Ctrl), hipHostMallocDefault));
        BFS_HIP(hipEventCreate(&w->ev_start));
        BFS_HIP(hipEventCreate(&w->ev_stop));
        BFS_HIP(hipEventCreateWithFlags(&w->ev_free, hipEventDisableTiming));
    } catch (...) {
        if (w->vis) (void)hipFree(w->vis);
        if (w->host_ctrl) (void)hipHostFree(w->host_ctrl);
        delete w;
        throw;
    }
    g->ws_all.push_back(w);
    g->device_bytes += w->bytes;
    if (t) *t = resolve_tunables(g, g->tun);
    ++g->ws_out;
    return w;
}

void release_ws(bfs_graph* g, Workspace* w, hipStream_t s) {
    if (hipEventRecord(w->ev_free, s) == hipSuccess) w->used = true;
    std::lock_guard<std::mutex> lk(g->mu);
    g->ws_free.push_back(w);
    --g->ws_out;
}

MsWorkspace* acquire_ms(bfs_graph* g, hipStream_t s, bfs_tunables* t) {
    std::lock_guard<std::mutex> lk(g->mu);
    MsWorkspace* w = nullptr;
    if (!g->ms_free.empty()) {
        w = g->ms_free.back();
        g->ms_free.pop_back();
        if (w->used) {
            const hipError_t e = hipStreamWaitEvent(s, w->ev_free, 0);
            if (e != hipSuccess) {
                g->ms_free.push_back(w);
                hip_check(e, "hipStreamWaitEvent");
            }
        }
        if (t) *t = resolve_tunables(g, g->tun);
        ++g->ws_out;
        return w;
    }
    w = new MsWorkspace();
    try {
        w->device = g->device;
        w->n = g->n;
        const size_t mb = (size_t)((g->n + 63) / 64 * 64) * 8;
        const size_t ctrl_bytes = (sizeof(MsCtrl) + 255) / 256 * 256 + 512;  // + join staging
        char* base = nullptr;
        BFS_HIP(hipMalloc(&base, mb * 3 + ctrl_bytes));
        w->vis = reinterpret_cast<unsigned long long*>(base);
        w->fr[0] = w->vis + mb / 8;
        w->fr[1] = w->fr[0] + mb / 8;
        w->ctrl = reinterpret_cast<MsCtrl*>(base + mb * 3);
        BFS_HIP(hipMemset(w->ctrl, 0, ctrl_bytes));
        BFS_HIP(hipHostMalloc(&w->host_ctrl, sizeof(MsCtrl), hipHostMallocDefault));
        BFS_HIP(hipEventCreate(&w->ev_start));
        BFS_HIP(hipEventCreate(&w->ev_stop));
        BFS_HIP(hipEventCreateWithFlags(&w->ev_free, hipEventDisableTiming));
        w->bytes = (int64_t)(mb * 3 + ctrl_bytes);
    } catch (...) {
        if (w->vis) (void)hipFree(w->vis);
        if (w->host_ctrl) (void)hipHostFree(w->host_ctrl);
        delete w;
        throw;
    }
    g->ms_all.push_back(w);
    g->device_bytes += w->bytes;
    if (t) *t = resolve_tunables(g, g->tun);
    ++g->ws_out;
    return w;
}

void release_ms(bfs_graph* g, MsWorkspace* w, hipStream_t s) {
    if (hipEventRecord(w->ev_free, s) == hipSuccess) w->used = true;
    std::lock_guard<std::mutex> lk(g->mu);
    g->ms_free.push_back(w);
    --g->ws_out;
}

void free_workspaces(bfs_graph* g) {
    for (Workspace* w : g->ws_all) {
        if (w->used) (void)hipEventSynchronize(w->ev_free);
        (void)hipFree(w->vis);
        if (w->out_levels) (void)hipFree(w->out_levels);
        (void)hipHostFree(w->host_ctrl);
        (void)hipEventDestroy(w->ev_start);
        (void)hipEventDestroy(w->ev_stop);
        (void)hipEventDestroy(w->ev_free);
        delete w;
    }
    for (MsWorkspace* w : g->ms_all) {
        if (w->used) (void)hipEventSynchronize(w->ev_free);
        (void)hipFree(w->vis);
        if (w->out_levels) (void)hipFree(w->out_levels);
        (void)hipHostFree(w->host_ctrl);
        (void)hipEventDestroy(w->ev_start);
        (void)hipEventDestroy(w->ev_stop);
        (void)hipEventDestroy(w->ev_free);
        delete w;
    }
    g->ws_all.clear();
    g->ws_free.clear();
    g->ms_all.clear();
    g->ms_free.clear();
}

// ---------------------------------------------------------------------------
// Load / free / info
// ---------------------------------------------------------------------------

bfs_graph* load_csr(int64_t n, int64_t nnz, const void* offsets, const int32_t* cols, uint32_t flags) {
    if (n < 1 || n > 2147483647LL) fail(BFS_E_INVALID_GRAPH, "n out of range");
    if (nnz < 0) fail(BFS_E_INVALID_GRAPH, "nnz < 0");
    if (nnz > 4294967295LL) fail(BFS_E_INVALID_GRAPH, "nnz above 2^32 - 1 (arc offsets of the big-row lists are 32-bit)");
    if (!offsets || (!cols && nnz > 0)) fail(BFS_E_INVALID_ARG, "NULL CSR array");
    if (flags & ~(BFS_LOAD_DEVICE_PTRS | BFS_LOAD_SKIP_VALIDATE | BFS_LOAD_OFFSETS_I32 | BFS_LOAD_SYMMETRIC))
        fail(BFS_E_INVALID_ARG, "unknown load flag");
    const bool dev = flags & BFS_LOAD_DEVICE_PTRS;
    const bool o32 = flags & BFS_LOAD_OFFSETS_I32;
    if (o32 && nnz > 2147483647LL) fail(BFS_E_INVALID_GRAPH, "nnz too large for int32 offsets");
    if (!(flags & BFS_LOAD_SKIP_VALIDATE) && !dev) {
        if (o32)
            validate_host(n, nnz, static_cast<const int32_t*>(offsets), cols);
        else
            validate_host(n, nnz, static_cast<const int64_t*>(offsets), cols);
    }
    bfs_graph* g = new bfs_graph();
    try {
        BFS_HIP(hipGetDevice(&g->device));
        g->cu_count = device_cu_count(g->device);
        g->n = n;
        g->nnz = nnz;
        g->off32 = o32;
        size_t ob = (size_t)(n + 1) * (o32 ? 4 : 8);
        if (dev) {
            if (!(flags & BFS_LOAD_SKIP_VALIDATE)) validate_device_csr(offsets, o32, cols, n, nnz);
            g->owns = false;
            g->d_off = const_cast<void*>(offsets);
            g->d_col = const_cast<int32_t*>(cols);
        } else {
            g->owns = true;
            BFS_HIP(hipMalloc(&g->d_off, ob));
            BFS_HIP(hipMalloc(&g->d_col, std::max<size_t>((size_t)nnz * 4, 4)));
            BFS_HIP(hipMemcpy(g->d_off, offsets, ob, hipMemcpyHostToDevice));
            if (nnz) BFS_HIP(hipMemcpy(g->d_col, cols, (size_t)nnz * 4, hipMemcpyHostToDevice));
            g->device_bytes += (int64_t)ob + nnz * 4;
        }
        if (flags & BFS_LOAD_SYMMETRIC) {
            if (!(flags & BFS_LOAD_SKIP_VALIDATE) && !csr_is_symmetric(g))
                fail(BFS_E_INVALID_GRAPH, "BFS_LOAD_SYMMETRIC: the arcs and the reversed arcs differ");
            g->symmetric = true;
            g->rows_sorted = csr_rows_sorted(g);
        }
        g->restore_grid = restore_grid_for(padded_words(n), g->cu_count);
        build_big_table(g->big, g->d_off, g->off32, n, default_tunables(nullptr).wave_max_degree, g->restore_grid,
                        g->cu_count, &g->max_degree);
        g->device_bytes += g->big.bytes;
        const bfs_tunables t = default_tunables(g);  // depends on the degrees just read
        build_hot_layout(g, hot_count(g, t), t.wave_max_degree, t.block_vertices);
        g->tun = t;
    } catch (...) {
        if (g->owns) {
            if (g->d_off) (void)hipFree(g->d_off);
            if (g->d_col) (void)hipFree(g->d_col);
        }
        free_big_table(g->big);
        free_hot_layout(g);
        delete g;
        throw;
    }
    return g;
}

void free_graph(bfs_graph* g) {
    if (g->server_refs.load() > 0) fail(BFS_E_BUSY, "graph is registered with a server");
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (g->ws_out > 0) fail(BFS_E_BUSY, "a run on this graph is in progress");
    }
    (void)hipDeviceSynchronize();
    free_workspaces(g);
    if (g->owns) {
        (void)hipFree(g->d_off);
        (void)hipFree(g->d_col);
    }
    free_big_table(g->big);
    free_hot_layout(g);
    delete g;
}

}  // namespace bfs
