// BFS server: the C ABI and the HIP engine of the scheduling core
// (serve_core.h). The core admits requests into multi-source instances,
// recycles their slots and pools result buffers; this engine runs the
// instances' levels on HIP streams (multi.hip) and the optional single-root
// runs with bfs_run.
#include <cstring>

#include "bfs_internal.h"
#include "serve_core.h"

namespace {

// Device side of one multi-source instance.
struct HipInstance {
    bfs::MsWorkspace* w = nullptr;
    bfs::MsCtrl* staging = nullptr;  // pinned slot table staging
    int32_t* join_stage = nullptr;   // pinned: slots and roots of one join
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;       // end of the level in flight
};

template <typename F>
auto device_call(F&& f) -> decltype(f()) {
    try {
        return f();
    } catch (const bfs::Error& e) {
        throw serve::EngineError(e.status, e.what());
    }
}

class HipEngine final : public serve::Engine {
   public:
    HipEngine(int device, int num_streams, int num_workers) : device_(device) {
        device_call([&] {
            for (int i = 0; i < num_streams; ++i) {
                hipStream_t st = nullptr;
                bfs::hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
                streams_.push_back(st);
            }
            for (int i = 0; i < num_workers; ++i) {
                hipStream_t st = nullptr;
                bfs::hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
                worker_streams_.push_back(st);
            }
        });
    }
    ~HipEngine() override {
        for (hipStream_t st : streams_) (void)hipStreamDestroy(st);
        for (hipStream_t st : worker_streams_) (void)hipStreamDestroy(st);
    }

    void thread_init() override {
        if (hipSetDevice(device_) != hipSuccess) throw serve::EngineError(BFS_E_DEVICE, "hipSetDevice");
    }
    int64_t graph_vertices(void* g) const override { return static_cast<bfs_graph*>(g)->n; }
    int64_t instance_bytes(void* g) const override {
        const int64_t n = static_cast<bfs_graph*>(g)->n;
        return ((n + 63) / 64 * 64) * 8 * 3 + (int64_t)sizeof(bfs::MsCtrl) + 1024;
    }
    void* alloc_result(int64_t bytes) override {
        void* b = nullptr;
        if (hipMalloc(&b, (size_t)bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return b;
    }
    void free_result(void* buf) override { (void)hipFree(buf); }

    void* create_instance(void* gp, int stream) override {
        return device_call([&] {
            bfs_graph* g = static_cast<bfs_graph*>(gp);
            auto in = std::make_unique<HipInstance>();
            in->stream = streams_[(size_t)stream];
            in->w = bfs::acquire_ms(g, in->stream);
            try {
                bfs::hip_check(hipHostMalloc(&in->staging, sizeof(bfs::MsCtrl), hipHostMallocDefault), "hipHostMalloc");
                std::memset(in->staging, 0, sizeof(bfs::MsCtrl));
                bfs::hip_check(hipHostMalloc(&in->join_stage, 128 * sizeof(int32_t), hipHostMallocDefault),
                               "hipHostMalloc");
                bfs::hip_check(hipEventCreateWithFlags(&in->done, hipEventDisableTiming), "hipEventCreate");
                bfs::ms_reset(g, in->w, in->stream);
                bfs::hip_check(hipStreamSynchronize(in->stream), "hipStreamSynchronize");
            } catch (...) {
                release(g, in.get());
                throw;
            }
            return static_cast<void*>(in.release());
        });
    }
    void destroy_instance(void* g, void* inst) override {
        HipInstance* in = static_cast<HipInstance*>(inst);
        release(static_cast<bfs_graph*>(g), in);
        delete in;
    }

    void join(void* gp, void* inst, const int32_t* slots, const int32_t* roots, void* const* bufs, int count,
              int level) override {
        device_call([&] {
            bfs_graph* g = static_cast<bfs_graph*>(gp);
            HipInstance* in = static_cast<HipInstance*>(inst);
            const int64_t n = g->n;
            for (int k = 0; k < count; ++k) {
                int32_t* buf = static_cast<int32_t*>(bufs[k]);
                bfs::launch_fill_i32(buf, 2 * n, -1, in->stream);
                bfs::ms_set_slot(in->w, in->staging, slots[k], buf, buf + n, level, in->stream);
            }
            bfs::ms_join(g, in->w, slots, roots, count, level, in->stream, in->join_stage);
        });
    }
    void step(void* gp, void* inst, int level) override {
        device_call([&] {
            bfs_graph* g = static_cast<bfs_graph*>(gp);
            HipInstance* in = static_cast<HipInstance*>(inst);
            const bfs_tunables t = bfs::current_tunables(g);
            bfs::ms_step_enqueue(g, t, in->w, level, in->stream, true);
            bfs::hip_check(hipEventRecord(in->done, in->stream), "hipEventRecord");
        });
    }
    bool ready(void* inst) override {
        const hipError_t e = hipEventQuery(static_cast<HipInstance*>(inst)->done);
        if (e == hipErrorNotReady) return false;
        device_call([&] { bfs::hip_check(e, "hipEventQuery"); });
        return true;
    }
    uint64_t alive(void* inst) override { return static_cast<HipInstance*>(inst)->w->host_ctrl->sum_alive; }
    void slot_totals(void* inst, int slot, int64_t* reached, int64_t* arcs) override {
        const bfs::MsCtrl* c = static_cast<HipInstance*>(inst)->w->host_ctrl;
        *reached = (int64_t)c->slot_reached[slot];
        *arcs = (int64_t)c->slot_arcs[slot];
    }
    void retire(void* g, void* inst, uint64_t keep) override {
        HipInstance* in = static_cast<HipInstance*>(inst);
        device_call([&] { bfs::ms_retire(static_cast<bfs_graph*>(g), in->w, keep, in->stream); });
    }
    int run_single(void* gp, int32_t root, void* buf, int worker, int32_t* levels, int64_t* reached,
                   int64_t* arcs) override {
        bfs_graph* g = static_cast<bfs_graph*>(gp);
        int32_t* b = static_cast<int32_t*>(buf);
        bfs_run_stats st{};
        const int rc = bfs_run(g, root, b, b + g->n, worker_streams_[(size_t)worker], 0, &st);
        *levels = st.num_levels;
        *reached = st.reached;
        *arcs = st.arcs_scanned;
        return rc;
    }
    int copy_out(void* buf, int64_t n, int32_t* levels, int32_t* parents) override {
        int rc = BFS_OK;
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (prev != device_) (void)hipSetDevice(device_);
        const int32_t* b = static_cast<const int32_t*>(buf);
        if (levels && hipMemcpy(levels, b, (size_t)n * 4, hipMemcpyDefault) != hipSuccess) rc = BFS_E_DEVICE;
        if (parents && hipMemcpy(parents, b + n, (size_t)n * 4, hipMemcpyDefault) != hipSuccess) rc = BFS_E_DEVICE;
        if (prev >= 0 && prev != device_) (void)hipSetDevice(prev);
        return rc;
    }
    void quiesce() override {
        (void)hipSetDevice(device_);
        for (hipStream_t st : streams_) (void)hipStreamSynchronize(st);
        for (hipStream_t st : worker_streams_) (void)hipStreamSynchronize(st);
    }

   private:
    static void release(bfs_graph* g, HipInstance* in) {
        if (in->w) bfs::release_ms(g, in->w, in->stream);
        if (in->staging) (void)hipHostFree(in->staging);
        if (in->join_stage) (void)hipHostFree(in->join_stage);
        if (in->done) (void)hipEventDestroy(in->done);
        in->w = nullptr;
        in->staging = nullptr;
        in->join_stage = nullptr;
        in->done = nullptr;
    }

    int device_;
    std::vector<hipStream_t> streams_;
    std::vector<hipStream_t> worker_streams_;
};

template <typename F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const bfs::Error& e) {
        return e.status;
    } catch (const serve::EngineError& e) {
        return e.status;
    } catch (const std::bad_alloc&) {
        return BFS_E_NO_MEMORY;
    } catch (...) {
        return BFS_E_INTERNAL;
    }
}

}  // namespace

struct bfs_server {
    int device = 0;
    std::unique_ptr<serve::Server> core;
    std::mutex mu;                   // guards graphs
    std::vector<bfs_graph*> graphs;  // registered graphs, for their server reference counts
};

extern "C" {

int bfs_server_create(const bfs_server_config* cfg, bfs_server** out) {
    return guarded([&] {
        if (!out) return BFS_E_INVALID_ARG;
        *out = nullptr;
        bfs_server_config c{};
        if (cfg) c = *cfg;
        if (c.flags != 0 || c.max_slots < 0 || c.max_slots > 64 || c.num_streams < 0 ||
            c.max_instances_per_graph < 0 || c.mem_budget_bytes < 0)
            return BFS_E_INVALID_ARG;
        if (c.max_slots == 0) c.max_slots = 64;
        // 16 streams keep a small graph's levels from queueing behind a large
        // graph's on a shared stream; 3 instances per graph let late arrivals
        // start without waiting for a busy instance's slots (8-graph Zipf
        // trace: p99 at 10k q/s 0.37 s against 0.49 s with 4 streams and 2).
        if (c.num_streams == 0) c.num_streams = 16;
        if (c.max_instances_per_graph == 0) c.max_instances_per_graph = 3;
        if (c.single_workers < -1 || c.batch_min_queue < 0) return BFS_E_INVALID_ARG;
        // Single-root workers are refused: a serving run that used them ended in
        // a GPU memory fault whose cause has not been found, so the route stays
        // closed until it has been.
        if (c.single_workers > 0) return BFS_E_INVALID_ARG;
        c.single_workers = 0;
        if (c.batch_min_queue == 0) c.batch_min_queue = 4;
        auto s = std::make_unique<bfs_server>();
        bfs::hip_check(hipGetDevice(&s->device), "hipGetDevice");
        if (c.mem_budget_bytes == 0) {
            size_t free_b = 0, total_b = 0;
            bfs::hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
            c.mem_budget_bytes = (int64_t)(free_b / 2);
        }
        auto eng = std::make_unique<HipEngine>(s->device, c.num_streams, c.single_workers);
        s->core = std::make_unique<serve::Server>(c, std::move(eng));
        *out = s.release();
        return BFS_OK;
    });
}

int bfs_server_add_graph(bfs_server* s, bfs_graph* g, int32_t* graph_id) {
    return guarded([&] {
        if (!s || !g || !graph_id) return BFS_E_INVALID_ARG;
        if (g->device != s->device) return BFS_E_INVALID_ARG;
        std::lock_guard<std::mutex> lk(s->mu);
        const int rc = s->core->add_graph(g, graph_id);
        if (rc == BFS_OK) {
            g->server_refs.fetch_add(1);
            s->graphs.push_back(g);
        }
        return rc;
    });
}

int bfs_server_submit(bfs_server* s, int32_t graph_id, int32_t root, uint64_t* ticket) {
    return guarded([&] {
        if (!s || !ticket) return BFS_E_INVALID_ARG;
        return s->core->submit(graph_id, root, ticket);
    });
}

int bfs_server_poll(bfs_server* s, uint64_t ticket, int32_t* levels, int32_t* parents, bfs_request_stats* st) {
    return guarded([&] {
        if (!s) return BFS_E_INVALID_ARG;
        return s->core->poll(ticket, levels, parents, st);
    });
}

int bfs_server_destroy(bfs_server* s) {
    return guarded([&] {
        if (!s) return BFS_OK;
        s->core.reset();  // stops the threads, waits for the device, frees instances and buffers
        for (bfs_graph* g : s->graphs) g->server_refs.fetch_sub(1);
        delete s;
        return BFS_OK;
    });
}

}  // extern "C"
