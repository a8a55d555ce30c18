// Deterministic predecessors for single-root runs (BFS_DETERMINISTIC).
//
// Any reached neighbour one layer up is a correct predecessor (section 3.2:
// the race between discoverers is benign), so a run's parents[] depends on the
// timing of its claims. The least such in-neighbour is a unique choice. After
// the levels are final, one pass replaces every parent by it:
//   * symmetric graphs: each reached vertex scans its own row (its
//     in-neighbours) for vertices one level up; with rows sorted by id the
//     first one found is the least and the scan stops there;
//   * other graphs: every reached u offers itself to each out-neighbour one
//     level down with atomicMin (the run's own parent is one of the offers).
// Both work on the caller's ids, levels and CSR.
#include <hip/hip_runtime.h>

#include <climits>

#include "bfs_internal.h"

namespace bfs {
namespace {

constexpr int kPassBlock = 256;
constexpr int kHeadArcs = 8;  // arcs a lane scans on its own before its wavefront helps

__device__ __forceinline__ int64_t shfl_i64(int64_t x, int src) {
    const int lo = __shfl((int)(uint32_t)(uint64_t)x, src, 64);
    const int hi = __shfl((int)(uint32_t)((uint64_t)x >> 32), src, 64);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Levels and parents were written by earlier kernels of the run, possibly on
// another XCD: read them with device-scope loads, as the run's own kernels do.
__device__ __forceinline__ int32_t ld_i32(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t wave_min_i32(int32_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const int32_t y = __shfl_xor(x, d, 64);
        x = y < x ? y : x;
    }
    return x;
}

// Symmetric graphs: parents[v] = least u in row v with levels[u] = levels[v] - 1.
// The run's own parent is such a u, so it starts as the best candidate and
// only smaller ids need a look: with sorted rows the scan ends at the first
// hit or at the first id not below the best.
template <typename OffT>
__global__ __launch_bounds__(kPassBlock) void k_least_parent_pull(const OffT* off, const int32_t* col,
                                                                  const int32_t* lv, int32_t* pa, int64_t n,
                                                                  int sorted) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * kPassBlock + threadIdx.x) >> 6;
    const int64_t waves = (int64_t)gridDim.x * (kPassBlock / 64);
    for (int64_t base = wave * 64; base < n; base += waves * 64) {
        const int64_t v = base + lane;
        const int L = v < n ? ld_i32(lv + v) : -1;
        const bool need = L > 0;  // reached and not the root
        int64_t b = 0, e = 0;
        int32_t best = INT_MAX;
        if (need) {
            b = (int64_t)off[v];
            e = (int64_t)off[v + 1];
            best = ld_i32(pa + v);
        }
        // The head of the row, its loads issued together.
        const int64_t head_end = e - b > kHeadArcs ? b + kHeadArcs : e;
        int32_t u[kHeadArcs];
        int lu[kHeadArcs];
#pragma unroll
        for (int k = 0; k < kHeadArcs; ++k) u[k] = b + k < head_end ? col[b + k] : INT_MAX;
#pragma unroll
        for (int k = 0; k < kHeadArcs; ++k) lu[k] = u[k] < best ? ld_i32(lv + u[k]) : -2;
        bool hit_head = false;
#pragma unroll
        for (int k = 0; k < kHeadArcs; ++k)
            if (lu[k] == L - 1 && u[k] < best) {
                best = u[k];
                hit_head = true;
            }
        bool done = !need || head_end == e || (sorted && (hit_head || u[kHeadArcs - 1] >= best));
        // Rows longer than the head: the wavefront scans 64 arcs at a time.
        uint64_t open = __ballot(!done);
        while (open) {
            const int src = __builtin_ctzll(open);
            open &= open - 1;
            const int64_t lb = shfl_i64(head_end, src), le = shfl_i64(e, src);
            const int want = __shfl(L, src, 64) - 1;
            int32_t m = __shfl(best, src, 64);
            for (int64_t j0 = lb; j0 < le; j0 += 64) {
                const int64_t j = j0 + lane;
                const int32_t x = j < le ? col[j] : INT_MAX;
                const bool hit = x < m && ld_i32(lv + x) == want;
                if (__ballot(hit)) {
                    const int32_t w = wave_min_i32(hit ? x : INT_MAX);
                    m = w < m ? w : m;
                    if (sorted) break;
                }
                if (sorted && !__ballot(x < m)) break;  // the rest of the row is not below the best
            }
            if (lane == src) best = m;
        }
        if (need) pa[v] = best;
    }
}

__device__ __forceinline__ void offer(int32_t* pa, int32_t v, int32_t u) {
    // A read filters offers that cannot lower the value (it only falls over
    // time, so an older value never hides a useful offer); the atomic decides.
    if (u < ld_i32(pa + v)) __hip_atomic_fetch_min(pa + v, u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Other graphs: every reached u offers itself to its out-neighbours one level
// down. Each parent starts as the run's own, which is one of the offers, so
// the minimum over the offers is the least parent.
template <typename OffT>
__global__ __launch_bounds__(kPassBlock) void k_least_parent_push(const OffT* off, const int32_t* col,
                                                                  const int32_t* lv, int32_t* pa, int64_t n) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * kPassBlock + threadIdx.x) >> 6;
    const int64_t waves = (int64_t)gridDim.x * (kPassBlock / 64);
    for (int64_t base = wave * 64; base < n; base += waves * 64) {
        const int64_t u = base + lane;
        const int L = u < n ? ld_i32(lv + u) : -1;
        int64_t b = 0, e = 0;
        if (L >= 0) {
            b = (int64_t)off[u];
            e = (int64_t)off[u + 1];
        }
        const int64_t head_end = e - b > kHeadArcs ? b + kHeadArcs : e;
        int32_t v[kHeadArcs];
        int lvv[kHeadArcs];
#pragma unroll
        for (int k = 0; k < kHeadArcs; ++k) v[k] = b + k < head_end ? col[b + k] : -1;
#pragma unroll
        for (int k = 0; k < kHeadArcs; ++k) lvv[k] = v[k] >= 0 ? ld_i32(lv + v[k]) : -2;
#pragma unroll
        for (int k = 0; k < kHeadArcs; ++k)
            if (lvv[k] == L + 1) offer(pa, v[k], (int32_t)u);
        uint64_t open = __ballot(head_end < e);
        while (open) {
            const int src = __builtin_ctzll(open);
            open &= open - 1;
            const int64_t lb = shfl_i64(head_end, src), le = shfl_i64(e, src);
            const int want = __shfl(L, src, 64) + 1;
            const int32_t us = (int32_t)shfl_i64(u, src);
            for (int64_t j0 = lb; j0 < le; j0 += 64) {
                const int64_t j = j0 + lane;
                if (j < le) {
                    const int32_t x = col[j];
                    if (ld_i32(lv + x) == want) offer(pa, x, us);
                }
            }
        }
    }
}

// Rows whose ids ever decrease (a count; 0 = every row sorted, ties allowed).
template <typename OffT>
__global__ __launch_bounds__(kPassBlock) void k_row_descents(const OffT* off, const int32_t* col, int64_t n,
                                                             unsigned long long* out) {
    const int64_t stride = (int64_t)gridDim.x * kPassBlock;
    unsigned long long c = 0;
    for (int64_t v = (int64_t)blockIdx.x * kPassBlock + threadIdx.x; v < n; v += stride) {
        const int64_t b = (int64_t)off[v], e = (int64_t)off[v + 1];
        for (int64_t j = b + 1; j < e; ++j)
            if (col[j] < col[j - 1]) {
                ++c;
                break;
            }
    }
    if (c) atomicAdd(out, c);
}

int pass_grid(const bfs_graph* g) {
    const int64_t want = (g->n + kPassBlock - 1) / kPassBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)g->cu_count * 16));
}

}  // namespace

void launch_least_parents(const bfs_graph* g, const int32_t* levels, int32_t* parents, hipStream_t s) {
    if (!levels || !parents) fail(BFS_E_INTERNAL, "no outputs for the parent pass");
    const int grid = pass_grid(g);
    if (g->symmetric) {
        if (g->off32)
            k_least_parent_pull<int32_t><<<grid, kPassBlock, 0, s>>>(static_cast<const int32_t*>(g->d_off), g->d_col,
                                                                     levels, parents, g->n, g->rows_sorted ? 1 : 0);
        else
            k_least_parent_pull<int64_t><<<grid, kPassBlock, 0, s>>>(static_cast<const int64_t*>(g->d_off), g->d_col,
                                                                     levels, parents, g->n, g->rows_sorted ? 1 : 0);
    } else {
        if (g->off32)
            k_least_parent_push<int32_t><<<grid, kPassBlock, 0, s>>>(static_cast<const int32_t*>(g->d_off), g->d_col,
                                                                     levels, parents, g->n);
        else
            k_least_parent_push<int64_t><<<grid, kPassBlock, 0, s>>>(static_cast<const int64_t*>(g->d_off), g->d_col,
                                                                     levels, parents, g->n);
    }
    BFS_HIP(hipGetLastError());
}

bool csr_rows_sorted(const bfs_graph* g) {
    unsigned long long* d = nullptr;
    unsigned long long h = 0;
    BFS_HIP(hipMalloc(&d, sizeof(h)));
    try {
        BFS_HIP(hipMemset(d, 0, sizeof(h)));
        const int grid = pass_grid(g);
        if (g->off32)
            k_row_descents<int32_t><<<grid, kPassBlock>>>(static_cast<const int32_t*>(g->d_off), g->d_col, g->n, d);
        else
            k_row_descents<int64_t><<<grid, kPassBlock>>>(static_cast<const int64_t*>(g->d_off), g->d_col, g->n, d);
        BFS_HIP(hipGetLastError());
        BFS_HIP(hipMemcpy(&h, d, sizeof(h), hipMemcpyDeviceToHost));
    } catch (...) {
        (void)hipFree(d);
        throw;
    }
    (void)hipFree(d);
    return h == 0;
}

}  // namespace bfs
