// Autotuner: coordinate descent over the kernel tunables on sample roots.
//
// Every candidate is timed with HIP events on a private stream (sum over the
// sample roots, best of two passes) and its levels are compared with those of
// the library defaults; a candidate that changes any level is rejected (the
// tunables only move work between bins, grids and update schemes, so this
// never happens unless something is broken). The winner is applied to the
// graph and returned.
#include <algorithm>
#include <cstring>
#include <vector>

#include "bfs_internal.h"

namespace bfs {

namespace {

struct Stream {
    hipStream_t s = nullptr;
    Stream() { hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate"); }
    ~Stream() { (void)hipStreamDestroy(s); }
};

struct DevBuf {
    int32_t* p = nullptr;
    explicit DevBuf(size_t count) { hip_check(hipMalloc(&p, std::max<size_t>(count, 1) * 4), "hipMalloc"); }
    ~DevBuf() { (void)hipFree(p); }
};

// Apply tunables to the graph (rebuilding derived tables when needed).
void apply(bfs_graph* g, const bfs_tunables& t) { apply_tunables(g, resolve_tunables(g, t)); }

// Time one candidate; fills `levels` (n per root, host) when not null.
double time_single(bfs_graph* g, const int32_t* roots, int count, hipStream_t s, int32_t* lv, int32_t* pa,
                   std::vector<int32_t>* levels) {
    const bfs_tunables t = current_tunables(g);
    hipEvent_t a, b;
    hip_check(hipEventCreate(&a), "hipEventCreate");
    hip_check(hipEventCreate(&b), "hipEventCreate");
    double best = 1e30;
    for (int pass = 0; pass < 2; ++pass) {
        double total = 0;
        for (int i = 0; i < count; ++i) {
            Workspace* w = acquire_ws(g, s);
            try {
                hip_check(hipEventRecord(a, s), "hipEventRecord");
                launch_single(g, t, w, roots[i], lv, pa, s);
                hip_check(hipEventRecord(b, s), "hipEventRecord");
                hip_check(hipEventSynchronize(b), "hipEventSynchronize");
            } catch (...) {
                release_ws(g, w, s);
                throw;
            }
            release_ws(g, w, s);
            float ms = 0;
            hip_check(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
            total += ms;
            if (levels && pass == 0) {
                hip_check(hipMemcpy(levels->data() + (size_t)i * g->n, lv, (size_t)g->n * 4, hipMemcpyDeviceToHost),
                          "hipMemcpy");
            }
        }
        best = std::min(best, total);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

double time_batch(bfs_graph* g, const int32_t* roots, int count, hipStream_t s, int32_t* lv, int32_t* pa,
                  std::vector<int32_t>* levels) {
    const bfs_tunables t = current_tunables(g);
    const int width = std::max(1, std::min(64, (int)t.batch_width));
    hipEvent_t a, b;
    hip_check(hipEventCreate(&a), "hipEventCreate");
    hip_check(hipEventCreate(&b), "hipEventCreate");
    double best = 1e30;
    for (int pass = 0; pass < 2; ++pass) {
        MsWorkspace* w = acquire_ms(g, s);
        try {
            hip_check(hipEventRecord(a, s), "hipEventRecord");
            for (int g0 = 0; g0 < count; g0 += width) {
                const int cnt = std::min(width, count - g0);
                ms_run_batch(g, t, w, roots + g0, cnt, lv + (int64_t)g0 * g->n, pa + (int64_t)g0 * g->n, g->n, s);
            }
            hip_check(hipEventRecord(b, s), "hipEventRecord");
            hip_check(hipEventSynchronize(b), "hipEventSynchronize");
        } catch (...) {
            release_ms(g, w, s);
            throw;
        }
        release_ms(g, w, s);
        float ms = 0;
        hip_check(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
        best = std::min(best, (double)ms);
        if (levels && pass == 0)
            hip_check(hipMemcpy(levels->data(), lv, (size_t)count * g->n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

}  // namespace

void autotune(bfs_graph* g, const int32_t* roots, int32_t num_roots, int32_t mode, bfs_tunables* best_out) {
    const int count = std::min<int32_t>(num_roots, mode == 0 ? 8 : 128);
    Stream st;
    const size_t rows = mode == 0 ? 1 : (size_t)count;
    DevBuf lv(rows * (size_t)g->n), pa(rows * (size_t)g->n);
    std::vector<int32_t> ref((size_t)count * g->n), got((size_t)count * g->n);

    auto measure = [&](const bfs_tunables& cand, bool reference) -> double {
        apply(g, cand);
        std::vector<int32_t>* out = reference ? &ref : &got;
        const double ms = mode == 0 ? time_single(g, roots, count, st.s, lv.p, pa.p, out)
                                    : time_batch(g, roots, count, st.s, lv.p, pa.p, out);
        if (!reference && got != ref) return 1e30;  // changed a level: rejected
        return ms;
    };

    bfs_tunables best = default_tunables(g);
    double best_ms = measure(best, true);

    struct Axis {
        int32_t bfs_tunables::*field;
        std::vector<int32_t> values;
    };
    std::vector<Axis> axes;
    if (mode == 0) {
        axes = {{&bfs_tunables::hot_vertices, {-1, 1 << 18, 1 << 19, 1 << 20}},
                {&bfs_tunables::block_size, {256, 512, 1024}},
                {&bfs_tunables::update_mode, {1, 2}},
                {&bfs_tunables::wave_max_degree, {64, 128, 256, 512, 1024}},
                {&bfs_tunables::small_max_degree, {8, 16, 32, 64, 256}},
                {&bfs_tunables::blocks_per_cu, {0, 2, 4}},
                {&bfs_tunables::block_vertices, {-1, 1 << 20}},
                {&bfs_tunables::sparse_frontier, {-1, 256, 1024, 4096}}};
        // The whole visited bitmap in LDS, where it fits beside every workgroup size.
        if (padded_words(g->n) <= std::min({lds_visited_words_max(256), lds_visited_words_max(512),
                                            lds_visited_words_max(1024)}))
            axes.insert(axes.begin() + 2, Axis{&bfs_tunables::lds_visited, {-1, 1}});
    } else {
        axes = {{&bfs_tunables::persistent, {1, -1}},
                {&bfs_tunables::batch_width, {16, 32, 64}},
                {&bfs_tunables::wave_max_degree, {128, 256, 1024}},
                {&bfs_tunables::small_max_degree, {16, 32, 64}},
                {&bfs_tunables::blocks_per_cu, {0, 2, 4}}};
    }
    for (int sweep = 0; sweep < 2; ++sweep) {
        bool improved = false;
        for (const Axis& ax : axes) {
            for (int32_t v : ax.values) {
                if (best.*(ax.field) == v) continue;
                bfs_tunables cand = best;
                cand.*(ax.field) = v;
                const double ms = measure(cand, false);
                if (ms < best_ms * 0.98) {  // keep a change only for a clear win
                    best_ms = ms;
                    best = resolve_tunables(g, cand);
                    improved = true;
                }
            }
        }
        if (!improved) break;
    }
    apply(g, best);
    if (best_out) *best_out = resolve_tunables(g, best);
}

}  // namespace bfs
