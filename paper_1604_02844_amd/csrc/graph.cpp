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
    return (int)std::max<int64_t>(1, std::min<int64_t>(chunks, (int64_t)std::max(cu_count, 1) * 8));
}

// Table of rows with degree > threshold (split over the whole expansion grid)
// and the bitmap that removes them from the per-wavefront frontier scan.
void rebuild_big(bfs_graph* g, int32_t threshold) {
    if (threshold < 1) threshold = 1;
    if (g->d_big && g->big_threshold == threshold) return;
    if (g->d_big) BFS_HIP(hipFree(g->d_big));
    if (g->d_big_prefix) BFS_HIP(hipFree(g->d_big_prefix));
    if (g->d_bigmap) BFS_HIP(hipFree(g->d_bigmap));
    if (g->d_seg_start) BFS_HIP(hipFree(g->d_seg_start));
    g->d_big = nullptr;
    g->d_big_prefix = nullptr;
    g->d_bigmap = nullptr;
    g->d_seg_start = nullptr;
    g->big_threshold = threshold;
    g->num_big = 0;
    g->big_arcs = 0;
    std::vector<int64_t> off((size_t)g->n + 1);
    if (g->off32) {
        std::vector<int32_t> o32((size_t)g->n + 1);
        BFS_HIP(hipMemcpy(o32.data(), g->d_off, o32.size() * 4, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < o32.size(); ++i) off[i] = o32[i];
    } else {
        BFS_HIP(hipMemcpy(off.data(), g->d_off, off.size() * 8, hipMemcpyDeviceToHost));
    }
    const int64_t words = padded_words(g->n);
    std::vector<uint32_t> bigmap((size_t)words, 0u);
    std::vector<int32_t> big;
    std::vector<int64_t> prefix(1, 0);
    g->max_degree = 0;
    for (int64_t v = 0; v < g->n; ++v) {
        const int64_t d = off[(size_t)v + 1] - off[(size_t)v];
        g->max_degree = std::max(g->max_degree, d);
        if (d > threshold) {
            big.push_back((int32_t)v);
            prefix.push_back(prefix.back() + d);
            bigmap[(size_t)(v >> 5)] |= 1u << (v & 31);
        }
    }
    g->num_big = (int32_t)big.size();
    g->big_arcs = prefix.back();
    BFS_HIP(hipMalloc(&g->d_big, std::max<size_t>(big.size(), 1) * 4));
    BFS_HIP(hipMalloc(&g->d_big_prefix, prefix.size() * 8));
    BFS_HIP(hipMalloc(&g->d_bigmap, (size_t)words * 4));
    if (!big.empty()) BFS_HIP(hipMemcpy(g->d_big, big.data(), big.size() * 4, hipMemcpyHostToDevice));
    BFS_HIP(hipMemcpy(g->d_big_prefix, prefix.data(), prefix.size() * 8, hipMemcpyHostToDevice));
    BFS_HIP(hipMemcpy(g->d_bigmap, bigmap.data(), (size_t)words * 4, hipMemcpyHostToDevice));
    // Segment capacities of the restore pass: the big rows inside the chunks
    // that each restore block visits.
    g->restore_grid = restore_grid_for(words, g->cu_count);
    std::vector<int32_t> seg((size_t)g->restore_grid + 1, 0);
    for (int64_t w = 0; w < words; ++w) {
        const int b = (int)((w / kRestoreBlock) % g->restore_grid);
        seg[(size_t)b + 1] += __builtin_popcount(bigmap[(size_t)w]);
    }
    for (int b = 0; b < g->restore_grid; ++b) seg[(size_t)b + 1] += seg[(size_t)b];
    BFS_HIP(hipMalloc(&g->d_seg_start, seg.size() * 4));
    BFS_HIP(hipMemcpy(g->d_seg_start, seg.data(), seg.size() * 4, hipMemcpyHostToDevice));
}

bfs_tunables default_tunables(const bfs_graph* g) {
    bfs_tunables t{};
    (void)g;
    t.small_max_degree = 32;
    t.wave_max_degree = 256;
    t.chunk_arcs = 0;
    t.block_size = 256;
    t.blocks_per_cu = 0;  // 0 = as many as fit (occupancy query at launch)
    t.batch_width = 64;
    t.update_mode = 1;
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
    if (t.block_size != 256 && t.block_size != 512) t.block_size = d.block_size;
    if (t.blocks_per_cu < 0) t.blocks_per_cu = 0;
    if (t.batch_width <= 0 || t.batch_width > 64) t.batch_width = d.batch_width;
    if (t.update_mode != 1 && t.update_mode != 2) t.update_mode = d.update_mode;
    return t;
}

// ---------------------------------------------------------------------------
// Workspace pools. A workspace returned to the pool records an event on the
// stream that used it; the next user on another stream waits for that event.
// ---------------------------------------------------------------------------

Workspace* acquire_ws(bfs_graph* g, hipStream_t s) {
    Workspace* w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (!g->ws_free.empty()) {
            w = g->ws_free.back();
            g->ws_free.pop_back();
        }
    }
    if (w) {
        if (w->used) BFS_HIP(hipStreamWaitEvent(s, w->ev_free, 0));
        return w;
    }
    w = new Workspace();
    try {
        w->device = g->device;
        w->words = padded_words(g->n);
        w->nslots = (int64_t)g->cu_count * 64 + 64;  // >= any expansion or restore grid
        w->big_capacity = std::max(g->num_big, 1);
        const size_t bmb = (size_t)w->words * 4;
        const size_t listb = (size_t)w->big_capacity * 8 + (size_t)(g->restore_grid + 1) * 8;
        const size_t total = bmb * 3 + sizeof(Ctrl) + (size_t)w->nslots * 2 * 8 + listb;
        char* base = nullptr;
        BFS_HIP(hipMalloc(&base, total));
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
        BFS_HIP(hipMemset(w->ctrl, 0, sizeof(Ctrl)));
        BFS_HIP(hipHostMalloc(&w->host_ctrl, sizeof(Ctrl), hipHostMallocDefault));
        BFS_HIP(hipEventCreate(&w->ev_start));
        BFS_HIP(hipEventCreate(&w->ev_stop));
        BFS_HIP(hipEventCreateWithFlags(&w->ev_free, hipEventDisableTiming));
        w->bytes = (int64_t)total;
    } catch (...) {
        if (w->vis) (void)hipFree(w->vis);
        if (w->host_ctrl) (void)hipHostFree(w->host_ctrl);
        delete w;
        throw;
    }
    std::lock_guard<std::mutex> lk(g->mu);
    g->ws_all.push_back(w);
    g->device_bytes += w->bytes;
    return w;
}

void release_ws(bfs_graph* g, Workspace* w, hipStream_t s) {
    if (hipEventRecord(w->ev_free, s) == hipSuccess) w->used = true;
    std::lock_guard<std::mutex> lk(g->mu);
    g->ws_free.push_back(w);
}

MsWorkspace* acquire_ms(bfs_graph* g, hipStream_t s) {
    MsWorkspace* w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (!g->ms_free.empty()) {
            w = g->ms_free.back();
            g->ms_free.pop_back();
        }
    }
    if (w) {
        if (w->used) BFS_HIP(hipStreamWaitEvent(s, w->ev_free, 0));
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
    std::lock_guard<std::mutex> lk(g->mu);
    g->ms_all.push_back(w);
    g->device_bytes += w->bytes;
    return w;
}

void release_ms(bfs_graph* g, MsWorkspace* w, hipStream_t s) {
    if (hipEventRecord(w->ev_free, s) == hipSuccess) w->used = true;
    std::lock_guard<std::mutex> lk(g->mu);
    g->ms_free.push_back(w);
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
    if (!offsets || (!cols && nnz > 0)) fail(BFS_E_INVALID_ARG, "NULL CSR array");
    if (flags & ~(BFS_LOAD_DEVICE_PTRS | BFS_LOAD_SKIP_VALIDATE | BFS_LOAD_OFFSETS_I32))
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
        g->tun = default_tunables(g);
        rebuild_big(g, g->tun.wave_max_degree);
        g->device_bytes += (int64_t)std::max(g->num_big, 1) * 4 + (int64_t)(g->num_big + 1) * 8 +
                           padded_words(n) * 4;
    } catch (...) {
        if (g->owns) {
            if (g->d_off) (void)hipFree(g->d_off);
            if (g->d_col) (void)hipFree(g->d_col);
        }
        if (g->d_big) (void)hipFree(g->d_big);
        if (g->d_big_prefix) (void)hipFree(g->d_big_prefix);
        if (g->d_bigmap) (void)hipFree(g->d_bigmap);
        if (g->d_seg_start) (void)hipFree(g->d_seg_start);
        delete g;
        throw;
    }
    return g;
}

void free_graph(bfs_graph* g) {
    if (g->server_refs.load() > 0) fail(BFS_E_BUSY, "graph is registered with a server");
    (void)hipDeviceSynchronize();
    free_workspaces(g);
    if (g->owns) {
        (void)hipFree(g->d_off);
        (void)hipFree(g->d_col);
    }
    if (g->d_big) (void)hipFree(g->d_big);
    if (g->d_big_prefix) (void)hipFree(g->d_big_prefix);
    if (g->d_bigmap) (void)hipFree(g->d_bigmap);
    if (g->d_seg_start) (void)hipFree(g->d_seg_start);
    delete g;
}

}  // namespace bfs
