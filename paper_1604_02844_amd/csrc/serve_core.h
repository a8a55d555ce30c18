// Scheduling core of the BFS server: continuous batching of single-root
// requests into multi-source instances. Host code only; every device action
// goes through an Engine, so the same core runs on the GPU (server.cpp, HIP
// engine) and on the CPU under thread and address sanitizers (a host engine in
// the tests).
//
// Requests (graph, root) are queued by submit from any thread. A scheduler
// thread owns every instance. Instances advance independently, each at its
// own pace on its own stream, so a request on a small graph never waits for a
// level of a large one:
//   admit   queued requests of a graph take free slots (bits) of one of that
//           graph's multi-source instances, when the memory budget has room
//           for their result rows; an instance is created on demand up to
//           max_instances_per_graph;
//   step    an instance that is not running a level seeds its newly admitted
//           roots and enqueues one level;
//   retire  when that level has completed, a slot whose bit is missing from
//           the next frontier has finished: its result rows go to the request,
//           its visited bits are cleared and the slot is free again.
// A new root joins with start level s = the instance level when it is seeded,
// so its vertices get instance level + 1 - s, i.e. its own hop distance: every
// request's result is the one a lone single-root BFS returns (levels exact,
// parents valid), whatever it was mixed with.
// Optional single-root workers take requests of lightly loaded graphs and
// serve each with one single-root run.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/bfs.h"

namespace serve {

using Clock = std::chrono::steady_clock;

inline double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// A failure of the device side, with the ABI status it maps to.
struct EngineError : std::runtime_error {
    int status;
    EngineError(int s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

// The device side. Graphs, instances and result buffers are opaque handles.
// Instance calls come from the scheduler thread only, run_single from the
// worker thread `worker`, copy_out from a polling thread; destroy calls come
// after those threads have stopped. Failures throw EngineError.
class Engine {
   public:
    virtual ~Engine() = default;
    virtual void thread_init() {}  // first call of the scheduler and worker threads
    virtual int64_t graph_vertices(void* g) const = 0;
    virtual int64_t instance_bytes(void* g) const = 0;  // budget charge of one instance
    virtual void* alloc_result(int64_t bytes) = 0;      // nullptr when none can be had now
    virtual void free_result(void* buf) = 0;
    virtual void* create_instance(void* g, int stream) = 0;
    virtual void destroy_instance(void* g, void* inst) = 0;
    // Seed `count` slots (result rows bufs[k]: levels[n] then parents[n]) at instance level `level`.
    virtual void join(void* g, void* inst, const int32_t* slots, const int32_t* roots, void* const* bufs, int count,
                      int level) = 0;
    virtual void step(void* g, void* inst, int level) = 0;  // enqueue one level
    virtual bool ready(void* inst) = 0;                     // the enqueued level has completed
    virtual uint64_t alive(void* inst) = 0;                 // slots with a next frontier (after ready)
    virtual void slot_totals(void* inst, int slot, int64_t* reached, int64_t* arcs) = 0;
    virtual void retire(void* g, void* inst, uint64_t keep) = 0;  // clear the visited bits of slots not in keep
    // One single-root run into buf; returns a status and the run's totals.
    virtual int run_single(void* g, int32_t root, void* buf, int worker, int32_t* levels, int64_t* reached,
                           int64_t* arcs) = 0;
    virtual int copy_out(void* buf, int64_t n, int32_t* levels, int32_t* parents) = 0;
    virtual void quiesce() = 0;  // wait for all enqueued device work
};

enum class ReqState { Queued, Running, Done, Failed };

struct Request {
    int32_t graph_id = 0;
    int32_t root = 0;
    ReqState state = ReqState::Queued;
    int status = BFS_OK;
    Clock::time_point t_submit, t_admit, t_done;
    void* buf = nullptr;  // result rows: levels[n] then parents[n]
    int32_t num_levels = 0;
    int64_t reached = 0, arcs = 0;
    bool batched = true;
};

struct Instance {
    void* h = nullptr;  // engine handle
    int stream = 0;
    bool in_flight = false;
    int level = 0;
    uint64_t slot_ticket[64] = {};
    int32_t slot_start[64] = {};
    uint64_t active = 0;  // slots running
    uint64_t used = 0;    // slots holding a request (running or joining)
    std::vector<int32_t> join_slots, join_roots;
    std::vector<void*> join_bufs;  // result rows of the joining slots
};

struct GraphState {
    void* g = nullptr;
    int64_t n = 0;
    std::deque<uint64_t> queue;
    std::vector<Instance*> inst;
    std::vector<void*> free_bufs;
};

class Server {
   public:
    // cfg must be resolved (no zero fields left to defaults); the server owns the engine.
    Server(const bfs_server_config& cfg, std::unique_ptr<Engine> eng) : cfg_(cfg), eng_(std::move(eng)) {
        stream_load_.assign((size_t)cfg_.num_streams, 0);
        idle_workers_ = cfg_.single_workers > 0 ? cfg_.single_workers : 0;
        thread_ = std::thread([this] { scheduler(); });
        try {
            for (int i = 0; i < cfg_.single_workers; ++i) workers_.emplace_back([this, i] { worker(i); });
        } catch (...) {
            stop_threads();
            throw;
        }
    }
    Server(const Server&) = delete;
    Server& operator=(const Server&) = delete;

    // Stops the threads, waits for the device, and frees every instance and buffer.
    ~Server() {
        stop_threads();
        try {
            eng_->quiesce();
        } catch (...) {
        }
        for (auto& gsp : graphs_) {
            GraphState& gs = *gsp;
            for (Instance* in : gs.inst) {
                try {
                    eng_->destroy_instance(gs.g, in->h);
                } catch (...) {
                }
                delete in;  // result rows of joining slots are freed with their requests below
            }
            for (void* b : gs.free_bufs) eng_->free_result(b);
        }
        for (auto& kv : reqs_)
            if (kv.second.buf) eng_->free_result(kv.second.buf);
    }

    int add_graph(void* g, int32_t* graph_id) {
        std::lock_guard<std::mutex> lk(mu_);
        if (stop_) return BFS_E_SHUTDOWN;
        auto gs = std::make_unique<GraphState>();
        gs->g = g;
        gs->n = eng_->graph_vertices(g);
        graphs_.push_back(std::move(gs));
        *graph_id = (int32_t)graphs_.size() - 1;
        return BFS_OK;
    }

    int submit(int32_t graph_id, int32_t root, uint64_t* ticket) {
        std::lock_guard<std::mutex> lk(mu_);
        if (stop_) return BFS_E_SHUTDOWN;
        if (fatal_) return fatal_;
        if (graph_id < 0 || graph_id >= (int32_t)graphs_.size()) return BFS_E_INVALID_ARG;
        GraphState& gs = *graphs_[(size_t)graph_id];
        if (root < 0 || root >= gs.n) return BFS_E_ROOT_RANGE;
        // A request must fit the budget on its own (instance plus result rows).
        if (eng_->instance_bytes(gs.g) + result_bytes(gs) > cfg_.mem_budget_bytes) return BFS_E_NO_MEMORY;
        const uint64_t t = next_ticket_++;
        Request r;
        r.graph_id = graph_id;
        r.root = root;
        r.t_submit = Clock::now();
        reqs_.emplace(t, r);
        gs.queue.push_back(t);
        *ticket = t;
        cv_.notify_one();
        return BFS_OK;
    }

    int poll(uint64_t ticket, int32_t* levels, int32_t* parents, bfs_request_stats* st) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return BFS_E_UNKNOWN_TICKET;
        Request& r = it->second;
        if (r.state == ReqState::Queued || r.state == ReqState::Running) return BFS_PENDING;
        GraphState& gs = *graphs_[(size_t)r.graph_id];
        if (r.state == ReqState::Failed) {
            const int status = r.status;
            // Result rows of a failed request go back to its graph's pool
            // (their contents are never read; a later request refills them).
            // A worker may still be writing them after a fatal error: the pool
            // then admits nobody any more, and destroy frees it after the
            // workers have stopped.
            if (r.buf) gs.free_bufs.push_back(r.buf);
            reqs_.erase(it);
            return status;
        }
        void* buf = r.buf;
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
        reqs_.erase(it);
        lk.unlock();
        // The result rows are complete (their level was observed complete).
        int rc = BFS_OK;
        try {
            rc = eng_->copy_out(buf, gs.n, levels, parents);
        } catch (const EngineError& e) {
            rc = e.status;
        }
        lk.lock();
        gs.free_bufs.push_back(buf);
        return rc;
    }

    // For tests: result and instance bytes charged against the budget.
    int64_t mem_used() {
        std::lock_guard<std::mutex> lk(mu_);
        return mem_used_;
    }

   private:
    void stop_threads() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        wcv_.notify_all();
        if (thread_.joinable()) thread_.join();
        for (auto& th : workers_) th.join();  // a worker finishes its run first
    }

    int64_t result_bytes(const GraphState& gs) const { return gs.n * 8; }

    // A result buffer (budget permitting) or nullptr. Caller holds mu_.
    void* take_buffer(GraphState& gs) {
        if (!gs.free_bufs.empty()) {
            void* b = gs.free_bufs.back();
            gs.free_bufs.pop_back();
            return b;
        }
        const int64_t need = result_bytes(gs);
        if (mem_used_ + need > cfg_.mem_budget_bytes) return nullptr;
        void* b = eng_->alloc_result(need);
        if (!b) return nullptr;
        mem_used_ += need;
        return b;
    }

    // Caller holds mu_.
    Instance* new_instance(GraphState& gs) {
        const int64_t need = eng_->instance_bytes(gs.g);
        if (mem_used_ + need > cfg_.mem_budget_bytes) return nullptr;
        if ((int)gs.inst.size() >= cfg_.max_instances_per_graph) return nullptr;
        // The stream carrying the fewest vertices of running instances: streams
        // map onto a few hardware queues, so keep small graphs away from large ones.
        size_t best = 0;
        for (size_t i = 1; i < stream_load_.size(); ++i)
            if (stream_load_[i] < stream_load_[best]) best = i;
        auto in = std::make_unique<Instance>();
        in->stream = (int)best;
        in->h = eng_->create_instance(gs.g, in->stream);
        stream_load_[best] += gs.n;
        gs.inst.push_back(in.get());
        mem_used_ += need;
        return in.release();
    }

    int free_slot(const Instance* in) const {
        for (int i = 0; i < cfg_.max_slots; ++i)
            if (!((in->used >> i) & 1ull)) return i;
        return -1;
    }

    // Admission at a level boundary. Caller holds mu_.
    void admit() {
        for (auto& gsp : graphs_) {
            GraphState& gs = *gsp;
            while (!gs.queue.empty()) {
                // While a graph's backlog is short, an idle single-root worker takes
                // the next request: one single-root run is cheaper than a
                // multi-source pass shared by few roots. A longer backlog goes to
                // the instances.
                if ((int)gs.queue.size() < cfg_.batch_min_queue && idle_workers_ > (int)single_queue_.size()) {
                    void* buf = take_buffer(gs);
                    if (!buf) break;
                    const uint64_t ticket = gs.queue.front();
                    gs.queue.pop_front();
                    Request& r = reqs_[ticket];
                    r.state = ReqState::Running;
                    r.t_admit = Clock::now();
                    r.buf = buf;
                    r.batched = false;
                    single_queue_.push_back(ticket);
                    wcv_.notify_one();
                    continue;
                }
                Instance* target = nullptr;
                int slot = -1;
                for (Instance* in : gs.inst) {
                    slot = free_slot(in);
                    if (slot >= 0) {
                        target = in;
                        break;
                    }
                }
                if (!target) {
                    target = new_instance(gs);
                    if (!target) break;  // no memory or instance limit: stays queued
                    slot = 0;
                }
                void* buf = take_buffer(gs);
                if (!buf) break;  // no room for the result rows yet
                const uint64_t ticket = gs.queue.front();
                gs.queue.pop_front();
                Request& r = reqs_[ticket];
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

    // A single-root worker: serves the requests routed to it, one run each.
    void worker(int index) {
        try {
            eng_->thread_init();
        } catch (...) {
            return;
        }
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            wcv_.wait(lk, [&] { return stop_ || !single_queue_.empty(); });
            if (stop_) return;
            const uint64_t ticket = single_queue_.front();
            single_queue_.pop_front();
            --idle_workers_;
            auto it = reqs_.find(ticket);
            if (it == reqs_.end() || it->second.state != ReqState::Running) {  // failed and consumed meanwhile
                ++idle_workers_;
                continue;
            }
            GraphState& gs = *graphs_[(size_t)it->second.graph_id];
            void* g = gs.g;
            const int32_t root = it->second.root;
            void* buf = it->second.buf;
            lk.unlock();
            int32_t nlev = 0;
            int64_t reached = 0, arcs = 0;
            int rc = BFS_OK;
            try {
                rc = eng_->run_single(g, root, buf, index, &nlev, &reached, &arcs);
            } catch (const EngineError& e) {
                rc = e.status;
            }
            const Clock::time_point now = Clock::now();
            lk.lock();
            ++idle_workers_;
            auto jt = reqs_.find(ticket);  // a running request cannot be consumed meanwhile
            if (jt != reqs_.end() && jt->second.state == ReqState::Running) {
                Request& r = jt->second;
                r.t_done = now;
                if (rc == BFS_OK) {
                    r.state = ReqState::Done;
                    r.num_levels = nlev;
                    r.reached = reached;
                    r.arcs = arcs;
                } else {
                    r.state = ReqState::Failed;
                    r.status = rc;
                }
            }
            cv_.notify_one();  // the scheduler may route more work here
        }
    }

    // Seed an idle instance's joining slots and enqueue its next level.
    void launch_step(GraphState& gs, Instance* in) {
        if (!in->join_slots.empty()) {
            for (int32_t slot : in->join_slots) in->slot_start[slot] = in->level;
            eng_->join(gs.g, in->h, in->join_slots.data(), in->join_roots.data(), in->join_bufs.data(),
                       (int)in->join_slots.size(), in->level);
            for (int32_t sl : in->join_slots) in->active |= 1ull << sl;
            in->join_slots.clear();
            in->join_roots.clear();
            in->join_bufs.clear();
        }
        eng_->step(gs.g, in->h, in->level);
        in->in_flight = true;
    }

    // The level in flight has completed: hand finished slots to their requests.
    void finish_step(GraphState& gs, Instance* in) {
        in->in_flight = false;
        const uint64_t alive = eng_->alive(in->h);
        const uint64_t finished = in->active & ~alive;
        if (finished) {
            const Clock::time_point now = Clock::now();
            std::lock_guard<std::mutex> lk(mu_);
            for (int i = 0; i < 64; ++i) {
                if (!((finished >> i) & 1ull)) continue;
                auto it = reqs_.find(in->slot_ticket[i]);
                if (it != reqs_.end()) {
                    Request& r = it->second;
                    r.state = ReqState::Done;
                    r.t_done = now;
                    r.num_levels = in->level - in->slot_start[i] + 1;
                    eng_->slot_totals(in->h, i, &r.reached, &r.arcs);
                }
                in->slot_ticket[i] = 0;
            }
            in->active &= ~finished;
            in->used &= ~finished;
            // Clear the finished slots' visited bits before their reuse.
            eng_->retire(gs.g, in->h, ~finished);
        }
        ++in->level;
    }

    void scheduler() {
        try {
            eng_->thread_init();
        } catch (const EngineError& e) {
            std::lock_guard<std::mutex> lk(mu_);
            fatal_ = e.status;
            fatal_msg_ = e.what();
        }
        std::vector<GraphState*> snapshot;
        bool progressed = true;
        while (true) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                bool busy = false, running = false;
                for (auto& gsp : graphs_) {
                    if (!gsp->queue.empty()) busy = true;
                    for (Instance* in : gsp->inst) {
                        if (in->active || !in->join_slots.empty()) busy = true;
                        if (in->in_flight) running = true;
                    }
                }
                if (!busy && !running && !stop_) cv_.wait_for(lk, std::chrono::milliseconds(2));
                if (stop_) return;
                if (fatal_) {  // nothing runs any more: wait for destroy
                    fail_all();
                    cv_.wait_for(lk, std::chrono::milliseconds(2));
                    continue;
                }
                try {
                    admit();
                } catch (const EngineError& e) {
                    fatal_ = e.status;
                    fatal_msg_ = e.what();
                }
                snapshot.clear();
                for (auto& gsp : graphs_) snapshot.push_back(gsp.get());
            }
            if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
            progressed = false;
            try {
                for (GraphState* gsp : snapshot) {
                    GraphState& gs = *gsp;
                    // gs.inst grows only in admit, on this thread.
                    for (Instance* in : gs.inst) {
                        if (in->in_flight) {
                            if (!eng_->ready(in->h)) continue;
                            finish_step(gs, in);
                            progressed = true;
                        }
                        if (!in->in_flight && (in->active || !in->join_slots.empty())) {
                            launch_step(gs, in);
                            progressed = true;
                        }
                    }
                }
            } catch (const EngineError& e) {
                std::lock_guard<std::mutex> lk(mu_);
                fatal_ = e.status;
                fatal_msg_ = e.what();
            }
        }
    }

    // After a device error: every queued or running request fails. Caller holds mu_.
    void fail_all() {
        for (auto& kv : reqs_)
            if (kv.second.state == ReqState::Queued || kv.second.state == ReqState::Running) {
                kv.second.state = ReqState::Failed;
                kv.second.status = fatal_;
            }
        for (auto& gsp : graphs_) gsp->queue.clear();
    }

    bfs_server_config cfg_;
    std::unique_ptr<Engine> eng_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::thread thread_;
    bool stop_ = false;
    std::vector<std::unique_ptr<GraphState>> graphs_;  // stable addresses
    std::unordered_map<uint64_t, Request> reqs_;
    uint64_t next_ticket_ = 1;
    std::vector<int64_t> stream_load_;  // vertices of the instances on each stream
    std::vector<std::thread> workers_;
    std::deque<uint64_t> single_queue_;
    std::condition_variable wcv_;
    int idle_workers_ = 0;
    int64_t mem_used_ = 0;
    int fatal_ = 0;  // a device error stops the scheduler; requests then fail
    std::string fatal_msg_;
};

}  // namespace serve
