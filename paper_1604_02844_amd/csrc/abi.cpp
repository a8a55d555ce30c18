// The C ABI of libbfs.so: argument checks, status mapping, and the host side of
// the single-root and batched runs. No C++ exception leaves these functions.
#include <algorithm>
#include <cstdio>
#include <cstring>

#include "bfs_internal.h"

namespace bfs {
bfs_graph* load_csr(int64_t n, int64_t nnz, const void* offsets, const int32_t* cols, uint32_t flags);
void free_graph(bfs_graph* g);
void autotune(bfs_graph* g, const int32_t* roots, int32_t num_roots, int32_t mode, bfs_tunables* best);
void run_noalloc(bfs_graph* g, int32_t root, int32_t* levels, int32_t* parents, hipStream_t s, bool hybrid);
}  // namespace bfs

namespace {

thread_local std::string g_last_error;

template <typename F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const bfs::Error& e) {
        g_last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return BFS_E_NO_MEMORY;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return BFS_E_INTERNAL;
    } catch (...) {
        g_last_error = "unknown exception";
        return BFS_E_INTERNAL;
    }
}

// Makes the graph's device current for the duration of a call.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) bfs::hip_check(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

void ensure_staging(bfs::Workspace* w, int64_t n) {
    if (w->out_levels) return;
    bfs::hip_check(hipMalloc(&w->out_levels, (size_t)n * 8), "hipMalloc staging");
    w->out_parents = w->out_levels + n;
}

void ensure_staging(bfs::MsWorkspace* w, int64_t n) {
    if (w->out_levels) return;
    bfs::hip_check(hipMalloc(&w->out_levels, (size_t)n * 64 * 8), "hipMalloc staging");
    w->out_parents = w->out_levels + n * 64;
}

}  // namespace

extern "C" {

const char* bfs_status_str(int status) {
    switch (status) {
        case BFS_OK: return "BFS_OK";
        case BFS_PENDING: return "BFS_PENDING";
        case BFS_E_INVALID_ARG: return "BFS_E_INVALID_ARG";
        case BFS_E_INVALID_GRAPH: return "BFS_E_INVALID_GRAPH";
        case BFS_E_ROOT_RANGE: return "BFS_E_ROOT_RANGE";
        case BFS_E_NO_MEMORY: return "BFS_E_NO_MEMORY";
        case BFS_E_DEVICE: return "BFS_E_DEVICE";
        case BFS_E_UNKNOWN_TICKET: return "BFS_E_UNKNOWN_TICKET";
        case BFS_E_BUSY: return "BFS_E_BUSY";
        case BFS_E_SHUTDOWN: return "BFS_E_SHUTDOWN";
        case BFS_E_INTERNAL: return "BFS_E_INTERNAL";
        default: return "BFS_E_UNKNOWN_STATUS";
    }
}

// Not part of bfs.h: the message of the calling thread's last error (for bindings).
const char* bfs_last_error(void) { return g_last_error.c_str(); }

int bfs_graph_load_csr(int64_t n, int64_t nnz, const void* offsets, const int32_t* cols, uint32_t flags,
                       bfs_graph** out) {
    return guarded([&] {
        if (!out) bfs::fail(BFS_E_INVALID_ARG, "out is NULL");
        *out = nullptr;
        *out = bfs::load_csr(n, nnz, offsets, cols, flags);
        return BFS_OK;
    });
}

int bfs_graph_free(bfs_graph* g) {
    return guarded([&] {
        if (!g) return BFS_OK;
        DeviceScope ds(g->device);
        bfs::free_graph(g);
        return BFS_OK;
    });
}

int bfs_graph_info(const bfs_graph* g, int64_t* n, int64_t* nnz, int64_t* device_bytes) {
    return guarded([&] {
        if (!g) bfs::fail(BFS_E_INVALID_ARG, "graph is NULL");
        if (n) *n = g->n;
        if (nnz) *nnz = g->nnz;
        if (device_bytes) *device_bytes = g->device_bytes;
        return BFS_OK;
    });
}

int bfs_graph_get_tunables(const bfs_graph* g, bfs_tunables* t) {
    return guarded([&] {
        if (!g || !t) bfs::fail(BFS_E_INVALID_ARG, "NULL argument");
        *t = bfs::current_tunables(const_cast<bfs_graph*>(g));
        return BFS_OK;
    });
}

int bfs_graph_set_tunables(bfs_graph* g, const bfs_tunables* t) {
    return guarded([&] {
        if (!g || !t) bfs::fail(BFS_E_INVALID_ARG, "NULL argument");
        DeviceScope ds(g->device);
        bfs::apply_tunables(g, bfs::resolve_tunables(g, *t));
        return BFS_OK;
    });
}

int bfs_run(bfs_graph* g, int32_t root, int32_t* levels, int32_t* parents, void* stream, uint32_t flags,
            bfs_run_stats* st) {
    return guarded([&] {
        if (!g || !levels || !parents) bfs::fail(BFS_E_INVALID_ARG, "NULL argument");
        if (flags & ~(BFS_OUT_HOST | BFS_ASYNC | BFS_HYBRID | BFS_DETERMINISTIC))
            bfs::fail(BFS_E_INVALID_ARG, "unknown run flag");
        const bool host_out = flags & BFS_OUT_HOST, async = flags & BFS_ASYNC, hybrid = flags & BFS_HYBRID;
        const bool least_parents = flags & BFS_DETERMINISTIC;
        if (async && (host_out || st)) bfs::fail(BFS_E_INVALID_ARG, "BFS_ASYNC excludes BFS_OUT_HOST and stats");
        if (root < 0 || root >= g->n) bfs::fail(BFS_E_ROOT_RANGE, "root out of range");
        if (hybrid && !g->symmetric) bfs::fail(BFS_E_INVALID_ARG, "BFS_HYBRID needs a graph loaded with BFS_LOAD_SYMMETRIC");
        DeviceScope ds(g->device);
        hipStream_t s = static_cast<hipStream_t>(stream);
        bfs_tunables t{};
        bfs::Workspace* w = bfs::acquire_ws(g, s, &t);
        try {
            int32_t* lv = levels;
            int32_t* pa = parents;
            if (host_out) {
                ensure_staging(w, g->n);
                lv = w->out_levels;
                pa = w->out_parents;
            }
            BFS_HIP(hipEventRecord(w->ev_start, s));
            if (least_parents) {
                bfs::launch_single(g, t, w, root, lv, pa, s, hybrid);
                bfs::launch_least_parents(g, lv, pa, s);
                BFS_HIP(hipEventRecord(w->ev_stop, s));
            } else {
                bfs::launch_single(g, t, w, root, lv, pa, s, hybrid, w->ev_stop);
            }
            if (host_out) {
                BFS_HIP(hipMemcpyAsync(levels, lv, (size_t)g->n * 4, hipMemcpyDeviceToHost, s));
                BFS_HIP(hipMemcpyAsync(parents, pa, (size_t)g->n * 4, hipMemcpyDeviceToHost, s));
            }
            if (st) {
                if (hybrid)
                    bfs::launch_single_stats_from_levels(g, t, w, lv, s);  // bottom-up levels scan no frontier rows
                else
                    bfs::launch_single_stats(w, s);
                BFS_HIP(hipMemcpyAsync(w->host_ctrl, w->ctrl, sizeof(bfs::Ctrl), hipMemcpyDeviceToHost, s));
            }
            if (!async) {
                BFS_HIP(hipStreamSynchronize(s));
                if (st) {
                    float ms = 0.f;
                    BFS_HIP(hipEventElapsedTime(&ms, w->ev_start, w->ev_stop));
                    st->num_levels = w->host_ctrl->num_levels;
                    st->num_roots = 1;
                    st->reached = (int64_t)w->host_ctrl->reached;
                    st->arcs_scanned = (int64_t)w->host_ctrl->arcs;
                    st->edges_traversed = st->arcs_scanned / 2;
                    st->device_ms = ms;
                }
            }
        } catch (...) {
            bfs::release_ws(g, w, s);
            throw;
        }
        bfs::release_ws(g, w, s);
        return BFS_OK;
    });
}

int bfs_run_noalloc(bfs_graph* g, int32_t root, int32_t* levels, int32_t* parents, void* stream, uint32_t flags) {
    return guarded([&] {
        if (!g || !levels || !parents) bfs::fail(BFS_E_INVALID_ARG, "NULL argument");
        if (flags & ~BFS_HYBRID) bfs::fail(BFS_E_INVALID_ARG, "bfs_run_noalloc takes BFS_HYBRID only");
        if (root < 0 || root >= g->n) bfs::fail(BFS_E_ROOT_RANGE, "root out of range");
        const bool hybrid = flags & BFS_HYBRID;
        if (hybrid && !g->symmetric) bfs::fail(BFS_E_INVALID_ARG, "BFS_HYBRID needs a graph loaded with BFS_LOAD_SYMMETRIC");
        DeviceScope ds(g->device);
        bfs::run_noalloc(g, root, levels, parents, static_cast<hipStream_t>(stream), hybrid);
        return BFS_OK;
    });
}

int bfs_run_batch(bfs_graph* g, const int32_t* roots, int32_t num_roots, int32_t* levels, int32_t* parents,
                  void* stream, uint32_t flags, bfs_run_stats* st) {
    return guarded([&] {
        if (!g || !roots || !levels || !parents) bfs::fail(BFS_E_INVALID_ARG, "NULL argument");
        if (num_roots < 1) bfs::fail(BFS_E_INVALID_ARG, "num_roots < 1");
        if (flags & ~(BFS_OUT_HOST | BFS_ASYNC)) bfs::fail(BFS_E_INVALID_ARG, "unknown run flag");
        const bool host_out = flags & BFS_OUT_HOST, async = flags & BFS_ASYNC;
        if (async && (host_out || st)) bfs::fail(BFS_E_INVALID_ARG, "BFS_ASYNC excludes BFS_OUT_HOST and stats");
        for (int32_t i = 0; i < num_roots; ++i)
            if (roots[i] < 0 || roots[i] >= g->n) bfs::fail(BFS_E_ROOT_RANGE, "root out of range");
        DeviceScope ds(g->device);
        hipStream_t s = static_cast<hipStream_t>(stream);
        bfs_tunables t{};
        bfs::MsWorkspace* w = bfs::acquire_ms(g, s, &t);
        const int width = std::max(1, std::min(64, (int)t.batch_width));
        int64_t reached = 0, arcs = 0;
        int32_t nlev = 0;
        double total_ms = 0;
        try {
            for (int32_t g0 = 0; g0 < num_roots; g0 += width) {
                const int32_t cnt = std::min<int32_t>(width, num_roots - g0);
                int32_t* lv = levels + (int64_t)g0 * g->n;
                int32_t* pa = parents + (int64_t)g0 * g->n;
                if (host_out) {
                    ensure_staging(w, g->n);
                    lv = w->out_levels;
                    pa = w->out_parents;
                }
                BFS_HIP(hipEventRecord(w->ev_start, s));
                // The stop event goes in after the batch's last kernel, before
                // the host's last wait when the batch ends as expected.
                bfs::ms_run_batch(g, t, w, roots + g0, cnt, lv, pa, g->n, s, w->ev_stop);
                if (host_out) {
                    BFS_HIP(hipMemcpyAsync(levels + (int64_t)g0 * g->n, lv, (size_t)cnt * g->n * 4,
                                           hipMemcpyDeviceToHost, s));
                    BFS_HIP(hipMemcpyAsync(parents + (int64_t)g0 * g->n, pa, (size_t)cnt * g->n * 4,
                                           hipMemcpyDeviceToHost, s));
                }
                // ms_run_batch has synchronised the stream and left the totals on the host.
                if (st) {
                    BFS_HIP(hipEventSynchronize(w->ev_stop));
                    float ms = 0.f;
                    BFS_HIP(hipEventElapsedTime(&ms, w->ev_start, w->ev_stop));
                    total_ms += ms;
                    reached += (int64_t)w->host_ctrl->total_disc;
                    arcs += (int64_t)w->host_ctrl->total_arcs;
                    nlev = std::max(nlev, w->host_ctrl->num_levels);
                }
            }
            if (!async) BFS_HIP(hipStreamSynchronize(s));
        } catch (...) {
            bfs::release_ms(g, w, s);
            throw;
        }
        bfs::release_ms(g, w, s);
        if (st) {
            st->num_levels = nlev;
            st->num_roots = num_roots;
            st->reached = reached;
            st->arcs_scanned = arcs;
            st->edges_traversed = arcs / 2;
            st->device_ms = total_ms;
        }
        return BFS_OK;
    });
}

int bfs_autotune(bfs_graph* g, const int32_t* roots, int32_t num_roots, int32_t mode, bfs_tunables* best) {
    return guarded([&] {
        if (!g || !roots || num_roots < 1) bfs::fail(BFS_E_INVALID_ARG, "bad autotune arguments");
        if (mode != 0 && mode != 1) bfs::fail(BFS_E_INVALID_ARG, "mode must be 0 or 1");
        for (int32_t i = 0; i < num_roots; ++i)
            if (roots[i] < 0 || roots[i] >= g->n) bfs::fail(BFS_E_ROOT_RANGE, "root out of range");
        DeviceScope ds(g->device);
        bfs::autotune(g, roots, num_roots, mode, best);
        return BFS_OK;
    });
}

}  // extern "C"
