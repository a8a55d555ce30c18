// BFS server: continuous batching of single-root requests into multi-source
// instances on resident graphs.
//
// Requests (graph, root) are queued by bfs_server_submit from any thread. A
// scheduler thread owns every device resource. Instances advance
// independently, each at its own pace on its own HIP stream, so a request on a
// small graph never waits for a level of a large one:
//   admit   queued requests of a graph take free slots (bits) of one of that
//           graph's multi-source instances, when the device-memory budget has
//           room for their result rows; an instance is created on demand up
//           to max_instances_per_graph;
//   step    an instance that is not running a level seeds its newly admitted
//           roots, enqueues one level and records an event;
//   retire  when that event has completed, a slot whose bit is missing from
//           the next frontier has finished: its result rows go to the request,
//           its visited bits are cleared and the slot is free again.
// A new root joins with start level s = the instance level when it is seeded,
// so its vertices get instance level + 1 - s, i.e. its own hop distance: every
// request's result is the one a lone single-root BFS returns (levels exact,
// parents valid), whatever it was mixed with.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include "bfs_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

enum class ReqState { Queued, Running, Done, Failed };

struct Request {
    int32_t graph_id = 0;
    int32_t root = 0;
    ReqState state = ReqState::Queued;
    int status = BFS_OK;
    Clock::time_point t_submit, t_admit, t_done;
    int32_t* buf = nullptr;  // device result rows: levels[n] then parents[n]
    int32_t num_levels = 0;
    int64_t reached = 0, arcs = 0;
    bool batched = true;
};

struct Instance {
    bfs::MsWorkspace* w = nullptr;
    bfs::MsCtrl* staging = nullptr;  // pinned slot table staging
    int32_t* join_stage = nullptr;   // pinned: slots and roots of one join
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;       // end of the level in flight
    bool in_flight = false;
    int level = 0;
    uint64_t slot_ticket[64] = {};
    int32_t slot_start[64] = {};
    uint64_t active = 0;  // slots running
    uint64_t used = 0;    // slots holding a request (running or joining)
    std::vector<int32_t> join_slots, join_roots;
    std::vector<int32_t*> join_bufs;  // result rows of the joining slots
};

struct GraphState {
    bfs_graph* g = nullptr;
    std::deque<uint64_t> queue;
    std::vector<Instance*> inst;
    std::vector<int32_t*> free_bufs;
};

}  // namespace

struct bfs_server {
    bfs_server_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::thread thread;
    bool stop = false;
    std::vector<std::unique_ptr<GraphState>> graphs;  // stable addresses
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    std::vector<hipStream_t> streams;
    std::vector<int64_t> stream_load;  // vertices of the instances on each stream
    // Single-root workers: requests of lightly loaded graphs, one bfs_run each.
    std::vector<std::thread> workers;
    std::vector<hipStream_t> worker_streams;
    std::deque<uint64_t> single_queue;
    std::condition_variable wcv;
    int idle_workers = 0;
    int64_t mem_used = 0;
    int fatal = 0;  // a device error stops the scheduler; requests then fail
    std::string fatal_msg;
};

namespace {

int64_t result_bytes(const bfs_graph* g) { return g->n * 8; }
int64_t instance_bytes(const bfs_graph* g) {
    return ((g->n + 63) / 64 * 64) * 8 * 3 + (int64_t)sizeof(bfs::MsCtrl) + 1024;
}

// Returns a result buffer (budget permitting) or nullptr. Caller holds mu.
int32_t* take_buffer(bfs_server* s, GraphState& gs) {
    if (!gs.free_bufs.empty()) {
        int32_t* b = gs.free_bufs.back();
        gs.free_bufs.pop_back();
        return b;
    }
    const int64_t need = result_bytes(gs.g);
    if (s->mem_used + need > s->cfg.mem_budget_bytes) return nullptr;
    int32_t* b = nullptr;
    if (hipMalloc(&b, (size_t)need) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    s->mem_used += need;
    return b;
}

Instance* new_instance(bfs_server* s, GraphState& gs) {
    const int64_t need = instance_bytes(gs.g);
    if (s->mem_used + need > s->cfg.mem_budget_bytes) return nullptr;
    if ((int)gs.inst.size() >= s->cfg.max_instances_per_graph) return nullptr;
    Instance* in = new Instance();
    // The stream carrying the fewest vertices of running instances: streams
    // map onto a few hardware queues, so keep small graphs away from large ones.
    size_t best = 0;
    for (size_t i = 1; i < s->streams.size(); ++i)
        if (s->stream_load[i] < s->stream_load[best]) best = i;
    s->stream_load[best] += gs.g->n;
    in->stream = s->streams[best];
    in->w = bfs::acquire_ms(gs.g, in->stream);
    bfs::hip_check(hipHostMalloc(&in->staging, sizeof(bfs::MsCtrl), hipHostMallocDefault), "hipHostMalloc");
    std::memset(in->staging, 0, sizeof(bfs::MsCtrl));
    bfs::hip_check(hipHostMalloc(&in->join_stage, 128 * sizeof(int32_t), hipHostMallocDefault), "hipHostMalloc");
    bfs::hip_check(hipEventCreateWithFlags(&in->done, hipEventDisableTiming), "hipEventCreate");
    bfs::ms_reset(gs.g, in->w, in->stream);
    bfs::hip_check(hipStreamSynchronize(in->stream), "hipStreamSynchronize");
    gs.inst.push_back(in);
    s->mem_used += need;
    return in;
}

int free_slot(const bfs_server* s, const Instance* in) {
    for (int i = 0; i < s->cfg.max_slots; ++i)
        if (!((in->used >> i) & 1ull)) return i;
    return -1;
}

// Admission at a level boundary. Caller holds mu.
void admit(bfs_server* s) {
    for (auto& gsp : s->graphs) {
        GraphState& gs = *gsp;
        while (!gs.queue.empty()) {
            // While a graph's backlog is short, an idle single-root worker takes
            // the next request: one bfs_run is cheaper than a multi-source pass
            // shared by few roots. A longer backlog goes to the instances.
            if ((int)gs.queue.size() < s->cfg.batch_min_queue && s->idle_workers > (int)s->single_queue.size()) {
                int32_t* buf = take_buffer(s, gs);
                if (!buf) break;
                const uint64_t ticket = gs.queue.front();
                gs.queue.pop_front();
                Request& r = s->reqs[ticket];
                r.state = ReqState::Running;
                r.t_admit = Clock::now();
                r.buf = buf;
                r.batched = false;
                s->single_queue.push_back(ticket);
                s->wcv.notify_one();
                continue;
            }
            Instance* target = nullptr;
            int slot = -1;
            for (Instance* in : gs.inst) {
                slot = free_slot(s, in);
                if (slot >= 0) {
                    target = in;
                    break;
                }
            }
            if (!target) {
                target = new_instance(s, gs);
                if (!target) break;  // no memory or instance limit: stays queued
                slot = 0;
            }
            int32_t* buf = take_buffer(s, gs);
            if (!buf) break;  // no room for the result rows yet
            const uint64_t ticket = gs.queue.front();
            gs.queue.pop_front();
            Request& r = s->reqs[ticket];
            r.state = ReqState::Running;
            r.t_admit = Clock::now();
            r.buf = buf;
            target->used |= 1ull << slot;
            target->slot_ticket[slot] = ticket;
            target->join_slots.push_back(slot);
            target->join_roots.push_back(r.root);
            target->join_bufs.push_back(buf);
        }
    }
}

// A single-root worker: runs bfs_run for requests routed to it, on its own stream.
void worker(bfs_server* s, int index) {
    if (hipSetDevice(s->device) != hipSuccess) return;
    hipStream_t stream = s->worker_streams[(size_t)index];
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        s->wcv.wait(lk, [&] { return s->stop || !s->single_queue.empty(); });
        if (s->stop) return;
        const uint64_t ticket = s->single_queue.front();
        s->single_queue.pop_front();
        --s->idle_workers;
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end() || it->second.state != ReqState::Running) {  // failed and consumed meanwhile
            ++s->idle_workers;
            continue;
        }
        bfs_graph* g = s->graphs[(size_t)it->second.graph_id]->g;
        const int32_t root = it->second.root;
        int32_t* buf = it->second.buf;
        lk.unlock();
        bfs_run_stats st{};
        const int rc = bfs_run(g, root, buf, buf + g->n, stream, 0, &st);
        const Clock::time_point now = Clock::now();
        lk.lock();
        ++s->idle_workers;
        auto jt = s->reqs.find(ticket);  // a running request cannot be consumed meanwhile
        if (jt != s->reqs.end() && jt->second.state == ReqState::Running) {
            Request& r = jt->second;
            r.t_done = now;
            if (rc == BFS_OK) {
                r.state = ReqState::Done;
                r.num_levels = st.num_levels;
                r.reached = st.reached;
                r.arcs = st.arcs_scanned;
            } else {
                r.state = ReqState::Failed;
                r.status = rc;
            }
        }
        s->cv.notify_one();  // the scheduler may route more work here
    }
}

// Seed an idle instance's joining slots and enqueue its next level.
void launch_step(GraphState& gs, Instance* in) {
    const int64_t n = gs.g->n;
    if (!in->join_slots.empty()) {
        for (size_t k = 0; k < in->join_slots.size(); ++k) {
            const int32_t slot = in->join_slots[k];
            int32_t* buf = in->join_bufs[k];
            in->slot_start[slot] = in->level;
            bfs::launch_fill_i32(buf, 2 * n, -1, in->stream);
            bfs::ms_set_slot(in->w, in->staging, slot, buf, buf + n, in->level, in->stream);
        }
        bfs::ms_join(gs.g, in->w, in->join_slots.data(), in->join_roots.data(), (int32_t)in->join_slots.size(),
                     in->level, in->stream, in->join_stage);
        for (int32_t sl : in->join_slots) in->active |= 1ull << sl;
        in->join_slots.clear();
        in->join_roots.clear();
        in->join_bufs.clear();
    }
    const bfs_tunables t = bfs::current_tunables(gs.g);
    bfs::ms_step_enqueue(gs.g, t, in->w, in->level, in->stream, true);
    bfs::hip_check(hipEventRecord(in->done, in->stream), "hipEventRecord");
    in->in_flight = true;
}

// The level in flight has completed: hand finished slots to their requests.
void finish_step(bfs_server* s, GraphState& gs, Instance* in) {
    in->in_flight = false;
    const uint64_t alive = in->w->host_ctrl->sum_alive;
    const uint64_t finished = in->active & ~alive;
    if (finished) {
        const Clock::time_point now = Clock::now();
        std::lock_guard<std::mutex> lk(s->mu);
        for (int i = 0; i < 64; ++i) {
            if (!((finished >> i) & 1ull)) continue;
            auto it = s->reqs.find(in->slot_ticket[i]);
            if (it != s->reqs.end()) {
                Request& r = it->second;
                r.state = ReqState::Done;
                r.t_done = now;
                r.num_levels = in->level - in->slot_start[i] + 1;
                r.reached = (int64_t)in->w->host_ctrl->slot_reached[i];
                r.arcs = (int64_t)in->w->host_ctrl->slot_arcs[i];
            }
            in->slot_ticket[i] = 0;
        }
        in->active &= ~finished;
        in->used &= ~finished;
        // Clear the finished slots' visited bits before their reuse.
        bfs::ms_retire(gs.g, in->w, ~finished, in->stream);
    }
    ++in->level;
}

void scheduler(bfs_server* s) {
    if (hipSetDevice(s->device) != hipSuccess) return;
    std::vector<GraphState*> snapshot;
    bool progressed = true;
    while (true) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            bool busy = false, running = false;
            for (auto& gsp : s->graphs) {
                if (!gsp->queue.empty()) busy = true;
                for (Instance* in : gsp->inst) {
                    if (in->active || !in->join_slots.empty()) busy = true;
                    if (in->in_flight) running = true;
                }
            }
            if (!busy && !running && !s->stop) s->cv.wait_for(lk, std::chrono::milliseconds(2));
            if (s->stop) return;
            if (s->fatal) {  // nothing runs any more: wait for bfs_server_destroy
                s->cv.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
            try {
                admit(s);
            } catch (const bfs::Error& e) {
                s->fatal = e.status;
                s->fatal_msg = e.what();
            }
            snapshot.clear();
            for (auto& gsp : s->graphs) snapshot.push_back(gsp.get());
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
        progressed = false;
        try {
            for (GraphState* gsp : snapshot) {
                GraphState& gs = *gsp;
                for (Instance* in : gs.inst) {
                    if (in->in_flight) {
                        const hipError_t e = hipEventQuery(in->done);
                        if (e == hipErrorNotReady) continue;
                        bfs::hip_check(e, "hipEventQuery");
                        finish_step(s, gs, in);
                        progressed = true;
                    }
                    if (!in->in_flight && (in->active || !in->join_slots.empty())) {
                        launch_step(gs, in);
                        progressed = true;
                    }
                }
            }
        } catch (const bfs::Error& e) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->fatal = e.status;
            s->fatal_msg = e.what();
        }
        if (s->fatal) {
            std::lock_guard<std::mutex> lk(s->mu);
            for (auto& kv : s->reqs)
                if (kv.second.state == ReqState::Queued || kv.second.state == ReqState::Running) {
                    kv.second.state = ReqState::Failed;
                    kv.second.status = s->fatal;
                }
            for (auto& gsp : s->graphs) gsp->queue.clear();
        }
    }
}

template <typename F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const bfs::Error& e) {
        return e.status;
    } catch (const std::bad_alloc&) {
        return BFS_E_NO_MEMORY;
    } catch (...) {
        return BFS_E_INTERNAL;
    }
}

}  // namespace

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
        auto* s = new bfs_server();
        bfs::hip_check(hipGetDevice(&s->device), "hipGetDevice");
        if (c.mem_budget_bytes == 0) {
            size_t free_b = 0, total_b = 0;
            bfs::hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
            c.mem_budget_bytes = (int64_t)(free_b / 2);
        }
        s->cfg = c;
        try {
            for (int i = 0; i < c.num_streams; ++i) {
                hipStream_t st = nullptr;
                bfs::hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
                s->streams.push_back(st);
                s->stream_load.push_back(0);
            }
            for (int i = 0; i < c.single_workers; ++i) {
                hipStream_t st = nullptr;
                bfs::hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
                s->worker_streams.push_back(st);
            }
            s->idle_workers = c.single_workers;
            s->thread = std::thread(scheduler, s);
            for (int i = 0; i < c.single_workers; ++i) s->workers.emplace_back(worker, s, i);
        } catch (...) {
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->stop = true;
            }
            s->cv.notify_all();
            s->wcv.notify_all();
            if (s->thread.joinable()) s->thread.join();
            for (auto& th : s->workers) th.join();
            for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
            for (hipStream_t st : s->worker_streams) (void)hipStreamDestroy(st);
            delete s;
            throw;
        }
        *out = s;
        return BFS_OK;
    });
}

int bfs_server_add_graph(bfs_server* s, bfs_graph* g, int32_t* graph_id) {
    return guarded([&] {
        if (!s || !g || !graph_id) return BFS_E_INVALID_ARG;
        if (g->device != s->device) return BFS_E_INVALID_ARG;
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return BFS_E_SHUTDOWN;
        auto gs = std::make_unique<GraphState>();
        gs->g = g;
        s->graphs.push_back(std::move(gs));
        g->server_refs.fetch_add(1);
        *graph_id = (int32_t)s->graphs.size() - 1;
        return BFS_OK;
    });
}

int bfs_server_submit(bfs_server* s, int32_t graph_id, int32_t root, uint64_t* ticket) {
    return guarded([&] {
        if (!s || !ticket) return BFS_E_INVALID_ARG;
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return BFS_E_SHUTDOWN;
        if (s->fatal) return s->fatal;
        if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size()) return BFS_E_INVALID_ARG;
        GraphState& gs = *s->graphs[(size_t)graph_id];
        if (root < 0 || root >= gs.g->n) return BFS_E_ROOT_RANGE;
        // A request must fit the budget on its own (instance plus result rows).
        if (instance_bytes(gs.g) + result_bytes(gs.g) > s->cfg.mem_budget_bytes) return BFS_E_NO_MEMORY;
        const uint64_t t = s->next_ticket++;
        Request r;
        r.graph_id = graph_id;
        r.root = root;
        r.t_submit = Clock::now();
        s->reqs.emplace(t, r);
        gs.queue.push_back(t);
        *ticket = t;
        s->cv.notify_one();
        return BFS_OK;
    });
}

int bfs_server_poll(bfs_server* s, uint64_t ticket, int32_t* levels, int32_t* parents, bfs_request_stats* st) {
    return guarded([&] {
        if (!s) return BFS_E_INVALID_ARG;
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return BFS_E_UNKNOWN_TICKET;
        Request& r = it->second;
        if (r.state == ReqState::Queued || r.state == ReqState::Running) return BFS_PENDING;
        if (r.state == ReqState::Failed) {
            const int status = r.status;
            // Result rows of a failed request go back to its graph's pool
            // (their contents are never read; a later request refills them).
            if (r.buf) s->graphs[(size_t)r.graph_id]->free_bufs.push_back(r.buf);
            s->reqs.erase(it);
            return status;
        }
        GraphState& gs = *s->graphs[(size_t)r.graph_id];
        const int64_t n = gs.g->n;
        int32_t* buf = r.buf;
        if (st) {
            st->num_levels = r.num_levels;
            st->graph_id = r.graph_id;
            st->reached = r.reached;
            st->arcs_scanned = r.arcs;
            st->edges_traversed = r.arcs / 2;
            st->queue_ms = ms_between(r.t_submit, r.t_admit);
            st->latency_ms = ms_between(r.t_submit, r.t_done);
            st->batched = r.batched ? 1 : 0;
            st->reserved = 0;
        }
        s->reqs.erase(it);
        lk.unlock();
        // The result rows are complete (the scheduler synchronised their stream).
        int rc = BFS_OK;
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (prev != s->device) (void)hipSetDevice(s->device);
        if (levels && hipMemcpy(levels, buf, (size_t)n * 4, hipMemcpyDefault) != hipSuccess) rc = BFS_E_DEVICE;
        if (parents && hipMemcpy(parents, buf + n, (size_t)n * 4, hipMemcpyDefault) != hipSuccess) rc = BFS_E_DEVICE;
        if (prev >= 0 && prev != s->device) (void)hipSetDevice(prev);
        lk.lock();
        gs.free_bufs.push_back(buf);
        return rc;
    });
}

int bfs_server_destroy(bfs_server* s) {
    return guarded([&] {
        if (!s) return BFS_OK;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv.notify_all();
        s->wcv.notify_all();
        if (s->thread.joinable()) s->thread.join();
        for (auto& th : s->workers) th.join();  // a worker finishes its bfs_run first
        (void)hipSetDevice(s->device);
        for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
        for (hipStream_t st : s->worker_streams) (void)hipStreamSynchronize(st);
        for (auto& gsp : s->graphs) {
            GraphState& gs = *gsp;
            for (Instance* in : gs.inst) {
                bfs::release_ms(gs.g, in->w, in->stream);
                (void)hipHostFree(in->staging);
                (void)hipHostFree(in->join_stage);
                (void)hipEventDestroy(in->done);
                delete in;  // result rows of joining slots are freed with their requests below
            }
            for (int32_t* b : gs.free_bufs) (void)hipFree(b);
            gs.g->server_refs.fetch_sub(1);
        }
        for (auto& kv : s->reqs)
            if (kv.second.buf) (void)hipFree(kv.second.buf);
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        for (hipStream_t st : s->worker_streams) (void)hipStreamDestroy(st);
        delete s;
        return BFS_OK;
    });
}

}  // extern "C"
