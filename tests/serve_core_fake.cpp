// The server's scheduling core (serve_core.h) driven by a host engine: each
// instance runs its multi-source levels on the CPU (a plain push level over 64
// root bits per vertex), completion shows up only after a random number of
// readiness queries, and single-root runs are plain queue BFS. Built with g++
// under ThreadSanitizer, and under AddressSanitizer with UndefinedBehavior-
// Sanitizer, by tests/test_serve_core_cpu.py. Every scenario checks each
// request's levels against an independent queue BFS, its parents (an arc from
// a vertex one level up), its totals, the buffer and instance accounting, and
// that destroy leaves no engine allocation behind.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <queue>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "serve_core.h"

namespace {

int g_failures = 0;
std::mutex g_fail_mu;

#define CHECK(cond, ...)                                              \
    do {                                                              \
        if (!(cond)) {                                                \
            std::lock_guard<std::mutex> lk_(g_fail_mu);               \
            ++g_failures;                                             \
            std::fprintf(stderr, "CHECK failed %s:%d: %s: ", __FILE__, __LINE__, #cond); \
            std::fprintf(stderr, __VA_ARGS__);                        \
            std::fprintf(stderr, "\n");                               \
        }                                                             \
    } while (0)

struct HostGraph {
    int64_t n = 0;
    std::vector<int64_t> off;
    std::vector<int32_t> col;
};

// Random symmetric graph: a path through every vertex of the first `reach`
// (so depths vary) plus random pairs; the rest may stay unreached.
HostGraph make_graph(int64_t n, int64_t pairs, int64_t reach, uint32_t seed) {
    std::mt19937 rng(seed);
    std::vector<std::pair<int32_t, int32_t>> e;
    for (int64_t v = 1; v < reach; ++v) e.emplace_back((int32_t)(v - 1), (int32_t)v);
    std::uniform_int_distribution<int64_t> pick(0, n - 1);
    for (int64_t i = 0; i < pairs; ++i) e.emplace_back((int32_t)pick(rng), (int32_t)pick(rng));
    HostGraph g;
    g.n = n;
    std::vector<std::vector<int32_t>> adj((size_t)n);
    for (auto& p : e) {
        if (p.first == p.second) continue;
        adj[(size_t)p.first].push_back(p.second);
        adj[(size_t)p.second].push_back(p.first);
    }
    g.off.assign((size_t)n + 1, 0);
    for (int64_t v = 0; v < n; ++v) g.off[(size_t)v + 1] = g.off[(size_t)v] + (int64_t)adj[(size_t)v].size();
    for (auto& a : adj) g.col.insert(g.col.end(), a.begin(), a.end());
    return g;
}

// Reference: plain FIFO queue BFS (levels; reached; arcs of reached rows).
std::vector<int32_t> ref_bfs(const HostGraph& g, int32_t root, int64_t* reached, int64_t* arcs) {
    std::vector<int32_t> lv((size_t)g.n, -1);
    std::queue<int32_t> q;
    lv[(size_t)root] = 0;
    q.push(root);
    *reached = 0;
    *arcs = 0;
    while (!q.empty()) {
        const int32_t u = q.front();
        q.pop();
        ++*reached;
        *arcs += g.off[(size_t)u + 1] - g.off[(size_t)u];
        for (int64_t j = g.off[(size_t)u]; j < g.off[(size_t)u + 1]; ++j) {
            const int32_t v = g.col[(size_t)j];
            if (lv[(size_t)v] < 0) {
                lv[(size_t)v] = lv[(size_t)u] + 1;
                q.push(v);
            }
        }
    }
    return lv;
}

struct FakeInstance {
    int64_t n = 0;
    std::vector<uint64_t> vis, fr, nfr;
    int32_t* out[64] = {};  // result rows of each slot
    int32_t start[64] = {};
    int64_t reached[64] = {}, arcs[64] = {};
    uint64_t alive = 0;
    int countdown = 0;  // readiness queries left before the level in flight completes
    bool in_flight = false;
};

class FakeEngine final : public serve::Engine {
   public:
    explicit FakeEngine(uint32_t seed, int fail_after_steps = -1) : rng_(seed), fail_after_(fail_after_steps) {}
    ~FakeEngine() override {
        std::lock_guard<std::mutex> lk(mu_);
        CHECK(live_bufs_.empty(), "%zu result buffers still allocated", live_bufs_.size());
        CHECK(live_inst_ == 0, "%d instances still allocated", live_inst_);
    }

    int64_t graph_vertices(void* g) const override { return static_cast<HostGraph*>(g)->n; }
    int64_t instance_bytes(void* g) const override { return static_cast<HostGraph*>(g)->n * 24 + 1024; }
    void* alloc_result(int64_t bytes) override {
        void* b = std::malloc((size_t)bytes);
        std::lock_guard<std::mutex> lk(mu_);
        live_bufs_.insert(b);
        return b;
    }
    void free_result(void* buf) override {
        std::lock_guard<std::mutex> lk(mu_);
        CHECK(live_bufs_.erase(buf) == 1, "free of an unknown result buffer");
        std::free(buf);
    }
    void* create_instance(void* g, int stream) override {
        CHECK(stream >= 0, "negative stream");
        auto* in = new FakeInstance();
        in->n = static_cast<HostGraph*>(g)->n;
        in->vis.assign((size_t)in->n, 0);
        in->fr.assign((size_t)in->n, 0);
        in->nfr.assign((size_t)in->n, 0);
        std::lock_guard<std::mutex> lk(mu_);
        ++live_inst_;
        return in;
    }
    void destroy_instance(void*, void* inst) override {
        delete static_cast<FakeInstance*>(inst);
        std::lock_guard<std::mutex> lk(mu_);
        --live_inst_;
    }
    void join(void* gp, void* inst, const int32_t* slots, const int32_t* roots, void* const* bufs, int count,
              int level) override {
        const HostGraph& g = *static_cast<HostGraph*>(gp);
        FakeInstance& in = *static_cast<FakeInstance*>(inst);
        CHECK(!in.in_flight, "join while a level is in flight");
        for (int k = 0; k < count; ++k) {
            const int s = slots[k];
            const int32_t r = roots[k];
            CHECK(s >= 0 && s < 64 && r >= 0 && r < g.n, "join slot %d root %d", s, r);
            CHECK(owned(bufs[k]), "join with a result buffer that is not allocated");
            int32_t* b = static_cast<int32_t*>(bufs[k]);
            std::fill(b, b + 2 * g.n, -1);
            in.out[s] = b;
            in.start[s] = level;
            const uint64_t bit = 1ull << s;
            CHECK(!(in.vis[(size_t)r] & bit), "slot %d reused with visited bits left", s);
            in.vis[(size_t)r] |= bit;
            in.fr[(size_t)r] |= bit;
            b[r] = 0;
            b[g.n + r] = r;
            in.reached[s] = 1;
            in.arcs[s] = g.off[(size_t)r + 1] - g.off[(size_t)r];
        }
    }
    void step(void* gp, void* inst, int level) override {
        if (fail_after_ >= 0 && steps_.fetch_add(1) >= fail_after_) throw serve::EngineError(BFS_E_DEVICE, "injected");
        const HostGraph& g = *static_cast<HostGraph*>(gp);
        FakeInstance& in = *static_cast<FakeInstance*>(inst);
        CHECK(!in.in_flight, "step while a level is in flight");
        // One push level: each root bit of a frontier row claims the unvisited heads.
        for (int64_t u = 0; u < g.n; ++u) {
            const uint64_t f = in.fr[(size_t)u];
            if (!f) continue;
            for (int64_t j = g.off[(size_t)u]; j < g.off[(size_t)u + 1]; ++j) {
                const int32_t v = g.col[(size_t)j];
                const uint64_t t = f & ~in.vis[(size_t)v];
                if (!t) continue;
                in.vis[(size_t)v] |= t;
                in.nfr[(size_t)v] |= t;
                for (uint64_t b = t; b; b &= b - 1) {
                    const int i = __builtin_ctzll(b);
                    CHECK(in.out[i] != nullptr, "discovery for slot %d without rows", i);
                    in.out[i][v] = level + 1 - in.start[i];
                    in.out[i][g.n + v] = (int32_t)u;
                }
            }
        }
        in.alive = 0;
        for (int64_t v = 0; v < g.n; ++v) {
            const uint64_t b = in.nfr[(size_t)v];
            in.fr[(size_t)v] = b;
            in.nfr[(size_t)v] = 0;
            in.alive |= b;
            for (uint64_t x = b; x; x &= x - 1) {
                const int i = __builtin_ctzll(x);
                ++in.reached[i];
                in.arcs[i] += g.off[(size_t)v + 1] - g.off[(size_t)v];
            }
        }
        std::lock_guard<std::mutex> lk(mu_);
        in.countdown = (int)(rng_() % 4);
        in.in_flight = true;
    }
    bool ready(void* inst) override {
        FakeInstance& in = *static_cast<FakeInstance*>(inst);
        CHECK(in.in_flight, "readiness query with nothing in flight");
        if (in.countdown > 0) {
            --in.countdown;
            return false;
        }
        in.in_flight = false;
        return true;
    }
    uint64_t alive(void* inst) override { return static_cast<FakeInstance*>(inst)->alive; }
    void slot_totals(void* inst, int slot, int64_t* reached, int64_t* arcs) override {
        const FakeInstance& in = *static_cast<FakeInstance*>(inst);
        *reached = in.reached[slot];
        *arcs = in.arcs[slot];
    }
    void retire(void*, void* inst, uint64_t keep) override {
        FakeInstance& in = *static_cast<FakeInstance*>(inst);
        for (auto& x : in.vis) x &= keep;
        for (int i = 0; i < 64; ++i)
            if (!((keep >> i) & 1ull)) in.out[i] = nullptr;
    }
    int run_single(void* gp, int32_t root, void* buf, int worker, int32_t* levels, int64_t* reached,
                   int64_t* arcs) override {
        CHECK(worker >= 0, "negative worker");
        CHECK(owned(buf), "single run into a result buffer that is not allocated");
        const HostGraph& g = *static_cast<HostGraph*>(gp);
        int32_t* b = static_cast<int32_t*>(buf);
        std::vector<int32_t> lv = ref_bfs(g, root, reached, arcs);
        std::fill(b, b + 2 * g.n, -1);
        int32_t maxl = 0;
        for (int64_t v = 0; v < g.n; ++v) {
            b[v] = lv[(size_t)v];
            maxl = std::max(maxl, lv[(size_t)v]);
            if (lv[(size_t)v] == 0) b[g.n + v] = root;
            if (lv[(size_t)v] > 0)
                for (int64_t j = g.off[(size_t)v]; j < g.off[(size_t)v + 1]; ++j)
                    if (lv[(size_t)g.col[(size_t)j]] == lv[(size_t)v] - 1) {
                        b[g.n + v] = g.col[(size_t)j];
                        break;
                    }
        }
        *levels = maxl + 1;
        return BFS_OK;
    }
    int copy_out(void* buf, int64_t n, int32_t* levels, int32_t* parents) override {
        CHECK(owned(buf), "copy from a result buffer that is not allocated");
        const int32_t* b = static_cast<const int32_t*>(buf);
        if (levels) std::memcpy(levels, b, (size_t)n * 4);
        if (parents) std::memcpy(parents, b + n, (size_t)n * 4);
        return BFS_OK;
    }
    void quiesce() override {}

   private:
    bool owned(void* b) {
        std::lock_guard<std::mutex> lk(mu_);
        return live_bufs_.count(b) == 1;
    }
    std::mutex mu_;
    std::mt19937 rng_;
    std::set<void*> live_bufs_;
    int live_inst_ = 0;
    int fail_after_;
    std::atomic<int> steps_{0};
};

bfs_server_config config(int64_t budget, int workers, int max_inst, int slots) {
    bfs_server_config c{};
    c.mem_budget_bytes = budget;
    c.max_slots = slots;
    c.num_streams = 4;
    c.max_instances_per_graph = max_inst;
    c.single_workers = workers;
    c.batch_min_queue = 4;
    return c;
}

void check_result(const HostGraph& g, int32_t root, const std::vector<int32_t>& lv, const std::vector<int32_t>& pa,
                  const bfs_request_stats& st, const char* what) {
    int64_t reached = 0, arcs = 0;
    const std::vector<int32_t> ref = ref_bfs(g, root, &reached, &arcs);
    int32_t maxl = 0;
    for (int64_t v = 0; v < g.n; ++v) {
        if (lv[(size_t)v] != ref[(size_t)v]) {
            CHECK(false, "%s: root %d vertex %lld level %d, expected %d", what, root, (long long)v, lv[(size_t)v],
                  ref[(size_t)v]);
            return;
        }
        maxl = std::max(maxl, ref[(size_t)v]);
        const int32_t p = pa[(size_t)v];
        if (ref[(size_t)v] < 0) {
            CHECK(p == -1, "%s: unreached vertex %lld has parent %d", what, (long long)v, p);
        } else if (v == root) {
            CHECK(p == root, "%s: root parent %d", what, p);
        } else {
            bool arc = false;
            if (p >= 0 && p < g.n && ref[(size_t)p] == ref[(size_t)v] - 1)
                for (int64_t j = g.off[(size_t)p]; j < g.off[(size_t)p + 1] && !arc; ++j) arc = g.col[(size_t)j] == v;
            CHECK(arc, "%s: root %d vertex %lld parent %d not one level up", what, root, (long long)v, p);
        }
    }
    CHECK(st.reached == reached && st.arcs_scanned == arcs && st.num_levels == maxl + 1,
          "%s: root %d totals %lld/%lld/%d, expected %lld/%lld/%d", what, root, (long long)st.reached,
          (long long)st.arcs_scanned, st.num_levels, (long long)reached, (long long)arcs, maxl + 1);
}

// Submitter threads each send requests over every graph, then poll all of them.
void mixed(const char* name, const std::vector<HostGraph>& graphs, bfs_server_config c, int threads, int per_thread) {
    auto eng = std::make_unique<FakeEngine>(7);
    {
        serve::Server s(c, std::move(eng));
        std::vector<int32_t> ids;
        for (const HostGraph& g : graphs) {
            int32_t id = -1;
            CHECK(s.add_graph(const_cast<HostGraph*>(&g), &id) == BFS_OK, "add_graph");
            ids.push_back(id);
        }
        std::vector<std::thread> th;
        for (int t = 0; t < threads; ++t)
            th.emplace_back([&, t] {
                std::mt19937 rng(100 + t);
                std::vector<std::pair<uint64_t, std::pair<int, int32_t>>> mine;
                for (int k = 0; k < per_thread; ++k) {
                    const int gi = (int)(rng() % graphs.size());
                    const int32_t root = (int32_t)(rng() % graphs[(size_t)gi].n);
                    uint64_t ticket = 0;
                    const int rc = s.submit(ids[(size_t)gi], root, &ticket);
                    CHECK(rc == BFS_OK, "%s: submit %d", name, rc);
                    if (rc == BFS_OK) mine.push_back({ticket, {gi, root}});
                    if (k % 7 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
                }
                for (auto& m : mine) {
                    const HostGraph& g = graphs[(size_t)m.second.first];
                    std::vector<int32_t> lv((size_t)g.n), pa((size_t)g.n);
                    bfs_request_stats st{};
                    int rc;
                    while ((rc = s.poll(m.first, lv.data(), pa.data(), &st)) == BFS_PENDING)
                        std::this_thread::sleep_for(std::chrono::microseconds(50));
                    CHECK(rc == BFS_OK, "%s: poll %d", name, rc);
                    if (rc == BFS_OK) check_result(g, m.second.second, lv, pa, st, name);
                    CHECK(s.poll(m.first, nullptr, nullptr, nullptr) == BFS_E_UNKNOWN_TICKET, "%s: ticket reused", name);
                }
            });
        for (auto& t : th) t.join();
        CHECK(s.mem_used() <= c.mem_budget_bytes, "%s: %lld bytes used over a budget of %lld", name,
              (long long)s.mem_used(), (long long)c.mem_budget_bytes);
    }
    std::printf("%s: %d requests ok\n", name, threads * per_thread);
}

// A device error after a few levels: every request fails with it, later
// submissions are refused with it, and destroy still frees everything.
void failure(const std::vector<HostGraph>& graphs) {
    auto eng = std::make_unique<FakeEngine>(9, 6);
    {
        serve::Server s(config(1 << 30, 0, 2, 64), std::move(eng));
        int32_t id = -1;
        CHECK(s.add_graph(const_cast<HostGraph*>(&graphs[0]), &id) == BFS_OK, "add_graph");
        std::vector<uint64_t> t;
        for (int k = 0; k < 40; ++k) {
            uint64_t ticket = 0;
            CHECK(s.submit(id, k % (int)graphs[0].n, &ticket) == BFS_OK, "submit");
            t.push_back(ticket);
        }
        int failed = 0, done = 0;
        for (uint64_t ticket : t) {
            int rc;
            while ((rc = s.poll(ticket, nullptr, nullptr, nullptr)) == BFS_PENDING)
                std::this_thread::sleep_for(std::chrono::microseconds(100));
            if (rc == BFS_E_DEVICE) ++failed;
            else if (rc == BFS_OK) ++done;
            else CHECK(false, "failure: poll returned %d", rc);
        }
        CHECK(failed > 0, "failure: no request failed");
        uint64_t ticket = 0;
        CHECK(s.submit(id, 0, &ticket) == BFS_E_DEVICE, "failure: submission after the error accepted");
        std::printf("failure: %d failed, %d done before the error\n", failed, done);
    }
}

// Destroy with requests queued, joining and running: nothing leaks.
void cancel(const std::vector<HostGraph>& graphs, int workers) {
    auto eng = std::make_unique<FakeEngine>(11);
    {
        serve::Server s(config(1 << 30, workers, 3, 64), std::move(eng));
        std::vector<int32_t> ids;
        for (const HostGraph& g : graphs) {
            int32_t id = -1;
            s.add_graph(const_cast<HostGraph*>(&g), &id);
            ids.push_back(id);
        }
        for (int k = 0; k < 300; ++k) {
            uint64_t ticket = 0;
            const HostGraph& g = graphs[(size_t)(k % graphs.size())];
            CHECK(s.submit(ids[(size_t)(k % graphs.size())], k % (int)g.n, &ticket) == BFS_OK, "submit");
        }
        std::this_thread::sleep_for(std::chrono::milliseconds(3));
    }
    std::printf("cancel (workers %d): destroyed with requests in flight\n", workers);
}

// Errors on bad arguments, before anything is queued.
void arguments(const std::vector<HostGraph>& graphs) {
    auto eng = std::make_unique<FakeEngine>(13);
    serve::Server s(config(1 << 30, 0, 1, 64), std::move(eng));
    int32_t id = -1;
    s.add_graph(const_cast<HostGraph*>(&graphs[0]), &id);
    uint64_t ticket = 0;
    CHECK(s.submit(id + 5, 0, &ticket) == BFS_E_INVALID_ARG, "unknown graph");
    CHECK(s.submit(id, (int32_t)graphs[0].n, &ticket) == BFS_E_ROOT_RANGE, "root out of range");
    CHECK(s.submit(id, -1, &ticket) == BFS_E_ROOT_RANGE, "negative root");
    CHECK(s.poll(12345, nullptr, nullptr, nullptr) == BFS_E_UNKNOWN_TICKET, "unknown ticket");
    std::printf("arguments ok\n");
}

}  // namespace

int main() {
    std::vector<HostGraph> graphs;
    graphs.push_back(make_graph(300, 400, 120, 1));   // deep path part, sparse
    graphs.push_back(make_graph(2000, 6000, 50, 2));
    graphs.push_back(make_graph(5000, 20000, 10, 3));
    graphs.push_back(make_graph(64, 0, 64, 4));       // a path: 64 levels
    // Room for one instance of the largest graph and two result rows: a second
    // request waits for a buffer, which comes back when a result is polled.
    // (Instances live as long as the server, so a budget that one graph's
    // instance fills would starve the other graphs: this case has one graph.)
    const HostGraph& largest = graphs[2];
    const int64_t tight = largest.n * 24 + 1024 + 2 * largest.n * 8;

    arguments(graphs);
    mixed("batched", graphs, config(1 << 30, 0, 3, 64), 4, 60);
    mixed("few slots", graphs, config(1 << 30, 0, 2, 3), 3, 40);
    // Budget for one instance of the largest graph and its result rows only:
    // admission waits for memory, results still arrive.
    mixed("tight budget", std::vector<HostGraph>{largest}, config(tight, 0, 3, 64), 3, 30);
    // The single-root route on the host engine (closed in the C ABI).
    mixed("workers", graphs, config(1 << 30, 3, 3, 64), 4, 60);
    failure(graphs);
    cancel(graphs, 0);
    cancel(graphs, 2);
    if (g_failures) {
        std::printf("FAILED: %d checks\n", g_failures);
        return 1;
    }
    std::printf("serve core: all scenarios ok\n");
    return 0;
}
