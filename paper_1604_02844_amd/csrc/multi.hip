// Multi-source BFS for gfx950: up to 64 independent BFS computed together,
// every vertex carrying a 64-bit visited mask and a 64-bit frontier mask (bit i
// belongs to root slot i).
//
// Each root follows the serial top-down method of the paper (section 3.1,
// Algorithm 1): a vertex of root i's current layer scans its neighbours, and a
// neighbour not yet visited by root i joins root i's next layer with level k+1
// and that vertex as parent. One pass over a row serves every root that has the
// row in its frontier. Per level the engine picks one of two directions, both
// of which give exactly the per-root layers of Algorithm 1:
//   push  (sparse frontiers) every frontier row u scans Adj[u]; for an arc
//         u->v the roots that claim v are t = frontier[u] & ~visited[v],
//         settled by a 64-bit atomicOr on visited[v] whose returned value
//         leaves each (root, vertex) pair one winner;
//   pull  (dense frontiers) every vertex v still missing some running root
//         gathers frontier[u] over Adj[v] until all missing bits are found;
//         the first neighbour providing a bit is that root's parent. Each v is
//         written by one lane only, so no atomics are needed — on gfx950 device
//         atomics run at about a tenth of the random-load rate.
// A finish pass then counts the next frontier (discoveries, arcs of its rows,
// OR of the slots still running), clears the consumed frontier buffer and, for
// the server, accumulates per-slot totals. Every statistic is striped over
// separate cache lines; the next level's kernels read the stripes and agree on
// the direction and on termination without host involvement.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>

#include "bfs_internal.h"

namespace bfs {

namespace {

typedef unsigned long long u64;

constexpr int kUnroll = 2;
constexpr int kPullUnroll = 8;
constexpr int kPullHead = 32;  // arcs a lane scans on its own before its wavefront helps
// Push while (arcs of the frontier rows) * alpha < nnz. A pull at an early
// dense level scans whole rows (few vertices find all their missing roots in
// one level), so it costs about nnz gathers, and a push arc (probe, atomicOr,
// record) about 4 gathers. Measured per batch (R-MAT 22 x64, ER 2^22 d16 x64
// and x8, ms): alpha 12: 10.1, 8.26, 3.49; 6: 10.1, 8.26, 2.97; 4: 7.37, 8.31,
// 3.01; 3: 7.34, 8.25, 3.28; 2: 7.40, 8.29, 3.33; 1: 21.4, 27.5, 5.86.
constexpr int kPushAlpha = 4;

// The slot table (output rows and start levels), copied into LDS by every
// workgroup of a level kernel, so that a discovery reads its row pointers
// from LDS instead of the control block.
struct SlotTable {
    int32_t* lv[64];
    int32_t* pa[64];
    int32_t start[64];
};

struct MsParams {
    const void* off;
    const int32_t* col;
    int32_t n;
    int64_t nnz;
    u64* vis;
    u64* fr;   // frontier of the level being expanded
    u64* nfr;  // next frontier
    MsCtrl* ctrl;
    const int32_t* big;
    const int64_t* big_prefix;
    const uint32_t* bigmap;
    int32_t num_big;
    int64_t big_arcs;
    int32_t t1;
    const SlotTable* slots;  // set inside the kernels to the LDS copy
};

// Shared state (masks, statistics, slot table) is accessed with device-scope
// loads and stores. Launch boundaries make the XCDs' L2 caches agree, so for
// state written only by earlier launches plain loads would do as well (the
// pull's neighbour masks read either way took the same time); within a launch
// each XCD's L2 does not see the others' stores, and device scope does.
template <typename T>
__device__ __forceinline__ T ld(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int rank_in(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

__device__ __forceinline__ int wave_incl_scan(int x, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ u64 shflu64(u64 x, int src) {
    int lo = __shfl((int)(uint32_t)x, src, 64);
    int hi = __shfl((int)(uint32_t)(x >> 32), src, 64);
    return ((u64)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ u64 shfl_xor_u64(u64 x, int mask) {
    int lo = __shfl_xor((int)(uint32_t)x, mask, 64);
    int hi = __shfl_xor((int)(uint32_t)(x >> 32), mask, 64);
    return ((u64)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ u64 wave_sum(u64 x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += shfl_xor_u64(x, d);
    return x;
}

__device__ __forceinline__ u64 wave_or(u64 x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x |= shfl_xor_u64(x, d);
    return x;
}

template <typename OffT>
__device__ __forceinline__ int64_t load_off(const void* off, int64_t i) {
    return (int64_t) static_cast<const OffT*>(off)[i];
}

__device__ __forceinline__ u64* sd(MsCtrl* c, int par, int s) { return &c->disc[par][s * kStripeStride]; }
__device__ __forceinline__ u64* sa(MsCtrl* c, int par, int s) { return &c->arcs[par][s * kStripeStride]; }
__device__ __forceinline__ u64* sl(MsCtrl* c, int par, int s) { return &c->alive[par][s * kStripeStride]; }
__device__ __forceinline__ u64* sw(MsCtrl* c, int s) { return &c->work[s * kStripeStride]; }

// Level summary read by every block of a level's kernels (same values everywhere).
struct LevelView {
    u64 disc, arcs, alive;
};

__device__ __forceinline__ LevelView read_level(MsCtrl* c, int lvl) {
    __shared__ u64 tmp[3];
    const int tid = threadIdx.x;
    if (tid < 64) {
        const int par = lvl & 1;
        const u64 d = wave_sum(ld(sd(c, par, tid)));
        const u64 a = wave_sum(ld(sa(c, par, tid)));
        const u64 l = wave_or(ld(sl(c, par, tid)));
        if (tid == 0) {
            tmp[0] = d;
            tmp[1] = a;
            tmp[2] = l;
        }
    }
    __syncthreads();
    LevelView v{tmp[0], tmp[1], tmp[2]};
    __syncthreads();
    return v;
}

__device__ __forceinline__ bool choose_push(const MsParams& p, const LevelView& v) {
    return (double)v.arcs * kPushAlpha < (double)p.nnz;
}

// Record the discovery of vertex v by the roots in nb, with parent u.
__device__ __forceinline__ void record(const SlotTable& t, int32_t v, int32_t u, u64 nb, int lvl) {
    while (nb) {
        const int i = __builtin_ctzll(nb);
        nb &= nb - 1;
        t.lv[i][v] = lvl + 1 - t.start[i];
        t.pa[i][v] = u;
    }
}

// Copy of the slot table into LDS (threads 0..63; the caller synchronises).
__device__ __forceinline__ void load_slots(MsCtrl* c, SlotTable& t) {
    const int i = threadIdx.x;
    if (i < 64) {
        t.lv[i] = ld(&c->out_lv[i]);
        t.pa[i] = ld(&c->out_pa[i]);
        t.start[i] = ld(&c->start[i]);
    }
}

// ---------------------------------------------------------------------------
// push
// ---------------------------------------------------------------------------

template <int U>
__device__ __forceinline__ void push_arcs(const MsParams& p, const int64_t (&pos)[U], const bool (&ok)[U],
                                          const int32_t (&par)[U], const u64 (&f)[U], int lvl) {
    int32_t v[U];
#pragma unroll
    for (int i = 0; i < U; ++i) v[i] = ok[i] ? __builtin_nontemporal_load(p.col + pos[i]) : 0;
    u64 t[U];
#pragma unroll
    for (int i = 0; i < U; ++i) t[i] = ok[i] ? (f[i] & ~p.vis[v[i]]) : 0ull;  // filter only
    u64 old[U];
#pragma unroll
    for (int i = 0; i < U; ++i) {
        old[i] = ~0ull;
        if (t[i]) old[i] = atomicOr(p.vis + v[i], t[i]);
    }
#pragma unroll
    for (int i = 0; i < U; ++i) {
        const u64 nb = t[i] & ~old[i];
        if (nb) {
            atomicOr(p.nfr + v[i], nb);
            record(*p.slots, v[i], par[i], nb, lvl);
        }
    }
}

template <int U>
__device__ __forceinline__ void push_row(const MsParams& p, int64_t beg, int64_t d, int32_t u, u64 f, int t,
                                         int nthreads, int lvl) {
    for (int64_t j0 = 0; j0 < d; j0 += (int64_t)nthreads * U) {
        int64_t pos[U];
        bool ok[U];
        int32_t par[U];
        u64 ff[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const int64_t j = j0 + (int64_t)i * nthreads + t;
            ok[i] = j < d;
            pos[i] = beg + j;
            par[i] = u;
            ff[i] = f;
        }
        push_arcs<U>(p, pos, ok, par, ff, lvl);
    }
}

template <typename OffT>
__device__ __forceinline__ void push_batch(const MsParams& p, int32_t u, u64 f, bool valid, int lane, int lvl) {
    int64_t beg = 0, d = 0;
    if (valid) {
        beg = load_off<OffT>(p.off, u);
        d = load_off<OffT>(p.off, (int64_t)u + 1) - beg;
    }
    const bool small = valid && d <= p.t1;
    const int ds = small ? (int)d : 0;
    const int incl = wave_incl_scan(ds, lane);
    const int excl = incl - ds;
    const int total = __shfl(incl, 63, 64);
    for (int base = 0; base < total; base += 64 * kUnroll) {
        int64_t pos[kUnroll];
        bool ok[kUnroll];
        int32_t par[kUnroll];
        u64 ff[kUnroll];
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) {
            const int a = base + i * 64 + lane;
            ok[i] = a < total;
            const int ac = ok[i] ? a : total - 1;
            int lo = 0, hi = 63;
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const int mid = (lo + hi) >> 1;
                if (__shfl(incl, mid, 64) > ac)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            const int ex = __shfl(excl, lo, 64);
            par[i] = __shfl(u, lo, 64);
            ff[i] = shflu64(f, lo);
            pos[i] = (int64_t)shflu64((u64)beg, lo) + (ac - ex);
        }
        push_arcs<kUnroll>(p, pos, ok, par, ff, lvl);
    }
    uint64_t mm = __ballot(valid && !small && d > 0);
    while (mm) {
        const int e = __builtin_ctzll(mm);
        mm &= mm - 1;
        push_row<kUnroll>(p, (int64_t)shflu64((u64)beg, e), (int64_t)shflu64((u64)d, e), __shfl(u, e, 64),
                          shflu64(f, e), lane, 64, lvl);
    }
}

template <int BLOCK>
struct PushShared {
    static constexpr int NW = BLOCK / 64;
    uint32_t ring_u[NW][128];
    u64 ring_f[NW][128];
    int32_t active[BLOCK];
    int nactive;
    int big_first;
};

// Start of level lvl, by every workgroup of its first kernel (or of the
// persistent batch kernel): the level's summary; workgroup 0 clears the next
// level's statistics and, when the frontier is empty, marks the run done.
__device__ __forceinline__ LevelView begin_level(const MsParams& p, int lvl) {
    const int tid = threadIdx.x;
    const LevelView lv = read_level(p.ctrl, lvl);
    if (blockIdx.x == 0 && tid < 64) {  // statistics of the next level start from zero
        const int np = (lvl + 1) & 1;
        st(sd(p.ctrl, np, tid), 0ull);
        st(sa(p.ctrl, np, tid), 0ull);
        st(sl(p.ctrl, np, tid), 0ull);
    }
    if (blockIdx.x == 0 && tid == 0) {
        if (lv.disc == 0) {
            st(&p.ctrl->num_levels, lvl);
            st(&p.ctrl->done, 1);
        } else {
            st(&p.ctrl->total_disc, ld(&p.ctrl->total_disc) + lv.disc);
            st(&p.ctrl->num_levels, lvl + 1);
        }
    }
    return lv;
}

// Push expansion of level lvl for the roots in `alive`, over the whole grid.
template <typename OffT, int BLOCK>
__device__ __forceinline__ void push_level(const MsParams& p, int lvl, u64 alive, PushShared<BLOCK>& sh) {
    constexpr int NW = BLOCK / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t G = gridDim.x, bid = blockIdx.x;

    // Rows of degree > T2: static split of their concatenated arcs.
    if (p.num_big > 0) {
        const int64_t per = (p.big_arcs + G - 1) / G;
        const int64_t s0 = bid * per;
        const int64_t s1 = s0 + per < p.big_arcs ? s0 + per : p.big_arcs;
        if (s0 < s1) {
            if (tid == 0) {
                int lo = 0, hi = p.num_big;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (p.big_prefix[mid + 1] > s0)
                        hi = mid;
                    else
                        lo = mid + 1;
                }
                sh.big_first = lo;
            }
            __syncthreads();
            for (int h0 = sh.big_first; h0 < p.num_big && p.big_prefix[h0] < s1; h0 += BLOCK) {
                if (tid == 0) sh.nactive = 0;
                __syncthreads();
                const int h = h0 + tid;
                if (h < p.num_big && p.big_prefix[h] < s1 && (ld(p.fr + p.big[h]) & alive))
                    sh.active[atomicAdd(&sh.nactive, 1)] = h;
                __syncthreads();
                const int na = sh.nactive;
                for (int i = 0; i < na; ++i) {
                    const int hh = sh.active[i];
                    const int64_t a0 = s0 > p.big_prefix[hh] ? s0 : p.big_prefix[hh];
                    const int64_t a1 = s1 < p.big_prefix[hh + 1] ? s1 : p.big_prefix[hh + 1];
                    const int32_t u = p.big[hh];
                    const int64_t beg = load_off<OffT>(p.off, u) + (a0 - p.big_prefix[hh]);
                    push_row<kUnroll>(p, beg, a1 - a0, u, ld(p.fr + u) & alive, tid, BLOCK, lvl);
                }
                __syncthreads();
            }
        }
    }

    // Other frontier rows: a contiguous run of 64-vertex tiles per wavefront.
    const int64_t tiles = ((int64_t)p.n + 63) / 64;
    const int64_t waves = G * NW;
    const int64_t gw = bid * NW + wid;
    const int64_t tpw = (tiles + waves - 1) / waves;
    const int64_t t0 = gw * tpw;
    const int64_t t1 = t0 + tpw < tiles ? t0 + tpw : tiles;
    uint32_t head = 0, tail = 0;
    for (int64_t ti = t0; ti < t1; ++ti) {
        const int64_t v = ti * 64 + lane;
        u64 f = 0;
        if (v < p.n && !((p.bigmap[v >> 5] >> (v & 31)) & 1u)) f = ld(p.fr + v) & alive;
        const bool has = f != 0;
        const uint64_t m = __ballot(has);
        if (has) {
            const uint32_t slot = (tail + rank_in(m)) & 127;
            sh.ring_u[wid][slot] = (uint32_t)v;
            sh.ring_f[wid][slot] = f;
        }
        tail += __popcll(m);
        if (tail - head >= 64) {
            const uint32_t slot = (head + lane) & 127;
            const int32_t u = (int32_t)sh.ring_u[wid][slot];
            const u64 fu = sh.ring_f[wid][slot];
            head += 64;
            push_batch<OffT>(p, u, fu, true, lane, lvl);
        }
    }
    if (tail != head) {
        const int cnt = (int)(tail - head);
        const bool valid = lane < cnt;
        const uint32_t slot = (head + lane) & 127;
        const int32_t u = valid ? (int32_t)sh.ring_u[wid][slot] : 0;
        const u64 fu = valid ? sh.ring_f[wid][slot] : 0ull;
        push_batch<OffT>(p, u, fu, valid, lane, lvl);
    }
}

template <typename OffT, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_ms_push(MsParams p, int lvl) {
    __shared__ PushShared<BLOCK> sh;
    __shared__ SlotTable slots;
    if (ld(&p.ctrl->done)) return;
    load_slots(p.ctrl, slots);  // synchronised by begin_level's barrier
    const LevelView lv = begin_level(p, lvl);
    if (lv.disc == 0 || !choose_push(p, lv)) return;
    p.slots = &slots;
    push_level<OffT, BLOCK>(p, lvl, lv.alive, sh);
}

// ---------------------------------------------------------------------------
// pull
// ---------------------------------------------------------------------------

// Exclusive prefix OR of x over the lanes below this one.
__device__ __forceinline__ u64 wave_excl_or(u64 x, int lane) {
    u64 incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int lo = __shfl_up((int)(uint32_t)incl, d, 64);
        const int hi = __shfl_up((int)(uint32_t)(incl >> 32), d, 64);
        if (lane >= d) incl |= ((u64)(uint32_t)hi << 32) | (uint32_t)lo;
    }
    const int lo = __shfl_up((int)(uint32_t)incl, 1, 64);
    const int hi = __shfl_up((int)(uint32_t)(incl >> 32), 1, 64);
    return lane == 0 ? 0ull : (((u64)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Each vertex still missing roots gathers its neighbours' frontier masks
// until every missing root is found. A lane scans the head of its own row;
// rows still open after it are scanned by the whole wavefront, 64 arcs at a
// time (coalesced column reads), so a hub row does not hold one lane for its
// whole length. A root bit found in several arcs of a step takes the lowest
// lane's neighbour as parent.
template <typename OffT>
__device__ __forceinline__ void pull_level(const MsParams& p, int lvl, u64 alive) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t base = wave * 64; base < p.n; base += waves * 64) {
        const int64_t v = base + lane;
        const bool valid = v < p.n;
        const u64 seen = valid ? ld(p.vis + v) : ~0ull;
        const u64 miss = alive & ~seen;
        u64 acc = 0;
        int64_t beg = 0, end = 0;
        if (miss) {
            beg = load_off<OffT>(p.off, v);
            end = load_off<OffT>(p.off, v + 1);
        }
        const int64_t head_end = end - beg > kPullHead ? beg + kPullHead : end;
        for (int64_t j = beg; j < head_end && acc != miss; j += kPullUnroll) {
            int32_t u[kPullUnroll];
            u64 f[kPullUnroll];
#pragma unroll
            for (int q = 0; q < kPullUnroll; ++q) u[q] = j + q < head_end ? p.col[j + q] : -1;
#pragma unroll
            for (int q = 0; q < kPullUnroll; ++q) f[q] = u[q] >= 0 ? ld(p.fr + u[q]) : 0ull;
#pragma unroll
            for (int q = 0; q < kPullUnroll; ++q) {
                const u64 nb = f[q] & miss & ~acc;
                if (nb) {
                    acc |= nb;
                    u64 b = nb;
                    while (b) {
                        const int i = __builtin_ctzll(b);
                        b &= b - 1;
                        p.slots->pa[i][v] = u[q];
                    }
                }
            }
        }
        // Rows still open: one at a time, by the whole wavefront.
        uint64_t open = __ballot(acc != miss && head_end < end);
        while (open) {
            const int src = __builtin_ctzll(open);
            open &= open - 1;
            const int64_t lb = (int64_t)shflu64((u64)head_end, src), le = (int64_t)shflu64((u64)end, src);
            const u64 m = shflu64(miss, src);
            const int32_t vs = (int32_t)(base + src);
            u64 a = shflu64(acc, src);
            for (int64_t j0 = lb; j0 < le && a != m; j0 += 64) {
                const int64_t j = j0 + lane;
                const bool in_row = j < le;
                const int32_t u = p.col[in_row ? j : le - 1];
                const u64 f = ld(p.fr + u);
                const u64 nb = in_row ? (f & m & ~a) : 0ull;
                const u64 mine = nb & ~wave_excl_or(nb, lane);
                for (u64 b = mine; b; b &= b - 1) p.slots->pa[__builtin_ctzll(b)][vs] = u;
                a |= wave_or(nb);
            }
            if (lane == src) acc = a;
        }
        if (valid) {
            st(p.nfr + v, acc);
            if (acc) {
                st(p.vis + v, seen | acc);
                u64 b = acc;
                while (b) {
                    const int i = __builtin_ctzll(b);
                    b &= b - 1;
                    p.slots->lv[i][v] = lvl + 1 - p.slots->start[i];
                }
            }
        }
    }
}

template <typename OffT>
__global__ __launch_bounds__(256) void k_ms_pull(MsParams p, int lvl) {
    __shared__ SlotTable slots;
    if (ld(&p.ctrl->done)) return;
    load_slots(p.ctrl, slots);  // synchronised by read_level's barrier
    const LevelView lview = read_level(p.ctrl, lvl);
    if (lview.disc == 0 || choose_push(p, lview)) return;
    p.slots = &slots;
    pull_level<OffT>(p, lvl, lview.alive);
}

// ---------------------------------------------------------------------------
// finish: statistics of the next frontier, clear the consumed frontier
// ---------------------------------------------------------------------------

template <typename OffT, bool kPerSlot>
__device__ __forceinline__ void finish_level(const MsParams& p, int lvl, u64 (&red)[4][4], u64* slot_r, u64* slot_a) {
    const int tid = threadIdx.x;
    if (kPerSlot) {
        if (tid < 64) {
            slot_r[tid] = 0;
            slot_a[tid] = 0;
        }
        __syncthreads();
    }
    u64 disc = 0, arcs = 0, alive = 0, work = 0;
    const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + tid; v < p.n; v += gsize) {
        const u64 b = ld(p.nfr + v);
        st(p.fr + v, 0ull);
        if (b) {
            const int64_t d = load_off<OffT>(p.off, v + 1) - load_off<OffT>(p.off, v);
            const int c = __popcll(b);
            disc += (u64)c;
            arcs += (u64)d;
            work += (u64)d * (u64)c;
            alive |= b;
            if (kPerSlot) {
                u64 x = b;
                while (x) {
                    const int i = __builtin_ctzll(x);
                    x &= x - 1;
                    atomicAdd(&slot_r[i], 1ull);
                    atomicAdd(&slot_a[i], (u64)d);
                }
            }
        }
    }
    disc = wave_sum(disc);
    arcs = wave_sum(arcs);
    work = wave_sum(work);
    alive = wave_or(alive);
    if ((tid & 63) == 0) {
        red[tid >> 6][0] = disc;
        red[tid >> 6][1] = arcs;
        red[tid >> 6][2] = alive;
        red[tid >> 6][3] = work;
    }
    __syncthreads();
    if (tid == 0) {
        u64 d = 0, a = 0, l = 0, wk = 0;
        for (int w = 0; w < 4; ++w) {
            d += red[w][0];
            a += red[w][1];
            l |= red[w][2];
            wk += red[w][3];
        }
        const int np = (lvl + 1) & 1;
        const int s = (int)(blockIdx.x % kStripes);
        if (d) {
            atomicAdd(sd(p.ctrl, np, s), d);
            atomicAdd(sa(p.ctrl, np, s), a);
            atomicOr(sl(p.ctrl, np, s), l);
            atomicAdd(sw(p.ctrl, s), wk);
        }
    }
    if (kPerSlot && tid < 64) {
        if (slot_r[tid]) atomicAdd(&p.ctrl->slot_reached[tid], slot_r[tid]);
        if (slot_a[tid]) atomicAdd(&p.ctrl->slot_arcs[tid], slot_a[tid]);
    }
}

template <typename OffT, bool kPerSlot>
__global__ __launch_bounds__(256) void k_ms_finish(MsParams p, int lvl) {
    __shared__ u64 red[4][4];
    __shared__ u64 slot_r[64], slot_a[64];
    if (ld(&p.ctrl->done)) return;
    finish_level<OffT, kPerSlot>(p, lvl, red, slot_r, slot_a);
}

// A whole batch in one cooperative launch (tunable persistent): every level's expansion (push or
// pull, chosen from the level summary that every workgroup reads alike) and
// its finish pass, separated by grid-wide barriers; the loop ends at the
// first empty frontier, the same level for every workgroup. The grid must be
// co-resident (the cooperative launch checks it), so no barrier waits for a
// workgroup that has not started.
template <typename OffT>
__global__ __launch_bounds__(256) void k_ms_batch(MsParams p, u64* fr0, u64* fr1, int max_levels) {
    __shared__ PushShared<256> sh;
    __shared__ u64 red[4][4];
    __shared__ SlotTable slots;
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    load_slots(p.ctrl, slots);  // synchronised by begin_level's barrier
    p.slots = &slots;
    for (int lvl = 0; lvl < max_levels; ++lvl) {
        p.fr = (lvl & 1) ? fr1 : fr0;
        p.nfr = (lvl & 1) ? fr0 : fr1;
        const LevelView lv = begin_level(p, lvl);
        if (lv.disc == 0) break;  // the same summary in every workgroup
        if (choose_push(p, lv))
            push_level<OffT, 256>(p, lvl, lv.alive, sh);
        else
            pull_level<OffT>(p, lvl, lv.alive);
        grid.sync();
        finish_level<OffT, false>(p, lvl, red, nullptr, nullptr);
        grid.sync();
    }
}

// After a batch: -1 level and parent for every (root, vertex) pair the batch
// did not reach (root i's bit absent from the vertex's visited mask). Every
// reached pair was written exactly once during the levels, so with this pass
// the output rows need no fill before the batch. Row i of the outputs starts
// at i * stride. Scattered pairs cost a line fetch each, so the pass is used
// only where few pairs stay unreached.
__global__ void k_ms_unreached(const u64* vis, int32_t* levels, int32_t* parents, int64_t stride, int count,
                               int64_t n) {
    const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
    const u64 all = count == 64 ? ~0ull : (1ull << count) - 1ull;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gsize) {
        const u64 m = ld(vis + v);
        if ((m & all) == all) continue;  // reached by every root of the batch
        for (int i = 0; i < count; ++i) {
            if (!((m >> i) & 1ull)) {
                levels[(int64_t)i * stride + v] = -1;
                parents[(int64_t)i * stride + v] = -1;
            }
        }
    }
}

__global__ void k_ms_clear(u64* vis, u64* a, u64* b, int64_t n) {
    const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gsize) {
        st(vis + v, 0ull);
        st(a + v, 0ull);
        st(b + v, 0ull);
    }
}

// Seed slots: root bits in visited and in the frontier of level `lvl`, level-0
// outputs, and the level's statistics.
template <typename OffT>
__global__ void k_ms_seed(MsParams p, const int32_t* slots, const int32_t* roots, int32_t count, int lvl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) st(&p.ctrl->done, 0);
    if (i >= count) return;
    const int s = slots[i];
    const int32_t r = roots[i];
    const u64 bit = 1ull << s;
    atomicOr(p.vis + r, bit);
    atomicOr(p.fr + r, bit);
    ld(&p.ctrl->out_lv[s])[r] = 0;
    ld(&p.ctrl->out_pa[s])[r] = r;
    const int64_t d = load_off<OffT>(p.off, (int64_t)r + 1) - load_off<OffT>(p.off, r);
    const int par = lvl & 1;
    atomicAdd(sd(p.ctrl, par, 0), 1ull);
    atomicAdd(sa(p.ctrl, par, 0), (u64)d);
    atomicOr(sl(p.ctrl, par, 0), bit);
    atomicAdd(sw(p.ctrl, 0), (u64)d);
    st(&p.ctrl->slot_reached[s], 1ull);
    st(&p.ctrl->slot_arcs[s], (u64)d);
}

__global__ void k_ms_summary(MsCtrl* c, int lvl) {
    const int tid = threadIdx.x;
    const int par = lvl & 1;
    const u64 d = wave_sum(ld(sd(c, par, tid)));
    const u64 a = wave_sum(ld(sa(c, par, tid)));
    const u64 l = wave_or(ld(sl(c, par, tid)));
    const u64 w = wave_sum(ld(sw(c, tid)));
    if (tid == 0) {
        st(&c->sum_disc, d);
        st(&c->sum_arcs, a);
        st(&c->sum_alive, l);
        st(&c->total_arcs, w);
    }
}

__global__ void k_ms_retire(u64* vis, int64_t n, u64 keep) {
    const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gsize) {
        const u64 x = ld(vis + v);
        if (x & ~keep) st(vis + v, x & keep);
    }
}

template <typename K>
int occupancy_of(K kernel, int block) {
    int occ = 0;
    hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, block, 0), "occupancy query");
    return occ;
}

MsParams make_params(bfs_graph* g, const bfs_tunables& t, MsWorkspace* w, int lvl) {
    MsParams p{};
    p.off = g->d_off;
    p.col = g->d_col;
    p.n = (int32_t)g->n;
    p.nnz = g->nnz;
    p.vis = w->vis;
    p.fr = w->fr[lvl & 1];
    p.nfr = w->fr[(lvl + 1) & 1];
    p.ctrl = w->ctrl;
    p.big = g->big.d_big;
    p.big_prefix = g->big.d_big_prefix;
    p.bigmap = g->big.d_bigmap;
    p.num_big = g->big.num_big;
    p.big_arcs = g->big.big_arcs;
    p.t1 = t.small_max_degree;
    return p;
}

int dense_grid(bfs_graph* g, int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, (int64_t)g->cu_count * 2));
}

template <typename OffT>
void enqueue_level(bfs_graph* g, const bfs_tunables& t, MsWorkspace* w, int lvl, bool per_slot, hipStream_t s) {
    if (g->big.threshold != t.wave_max_degree) fail(BFS_E_INTERNAL, "big-row table out of date");
    MsParams p = make_params(g, t, w, lvl);
    static const int occ = occupancy_of(k_ms_push<OffT, 256>, 256);
    // On gfx950 one workgroup per CU fewer than the occupancy query reports is
    // resident at once (measured: with the reported count, one workgroup per CU
    // starts only when another finishes); a grid that fits keeps every
    // workgroup's share in the first wave of the dispatch.
    const int fit = occ > 1 ? occ - 1 : 1;
    const int bpc = t.blocks_per_cu > 0 && t.blocks_per_cu < fit ? t.blocks_per_cu : fit;
    const int push_grid = bpc * g->cu_count;
    const int pull_grid = (int)std::max<int64_t>(1, std::min<int64_t>((g->n + 255) / 256, (int64_t)g->cu_count * 8));
    const int dg = dense_grid(g, g->n);
    k_ms_push<OffT, 256><<<push_grid, 256, 0, s>>>(p, lvl);
    k_ms_pull<OffT><<<pull_grid, 256, 0, s>>>(p, lvl);
    if (per_slot)
        k_ms_finish<OffT, true><<<dg, 256, 0, s>>>(p, lvl);
    else
        k_ms_finish<OffT, false><<<dg, 256, 0, s>>>(p, lvl);
    BFS_HIP(hipGetLastError());
}

// One cooperative launch of the persistent batch kernel: at most
// (occupancy - 1) workgroups per CU (one fewer than the occupancy query
// reports is what stays resident on gfx950), fewer with blocks_per_cu; the
// cooperative launch refuses a grid that cannot be co-resident.
template <typename OffT>
void launch_batch_persistent(bfs_graph* g, const bfs_tunables& t, MsWorkspace* w, hipStream_t s) {
    if (g->big.threshold != t.wave_max_degree) fail(BFS_E_INTERNAL, "big-row table out of date");
    MsParams p = make_params(g, t, w, 0);
    static const int occ = occupancy_of(k_ms_batch<OffT>, 256);
    const int fit = occ > 1 ? occ - 1 : 1;
    const int bpc = t.blocks_per_cu > 0 && t.blocks_per_cu < fit ? t.blocks_per_cu : fit;
    const int grid = bpc * g->cu_count;
    if (grid < 1 || grid > occ * g->cu_count) fail(BFS_E_INTERNAL, "persistent grid larger than the resident set");
    int max_levels = (int)std::min<int64_t>(g->n + 1, (int64_t)INT32_MAX);
    unsigned long long* fr0 = w->fr[0];
    unsigned long long* fr1 = w->fr[1];
    void* args[] = {&p, &fr0, &fr1, &max_levels};
    BFS_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_ms_batch<OffT>), dim3(grid), dim3(256), args,
                                       0, s));
}

void enqueue_level_any(bfs_graph* g, const bfs_tunables& t, MsWorkspace* w, int lvl, bool per_slot, hipStream_t s) {
    if (g->off32)
        enqueue_level<int32_t>(g, t, w, lvl, per_slot, s);
    else
        enqueue_level<int64_t>(g, t, w, lvl, per_slot, s);
}

}  // namespace

void ms_reset(bfs_graph* g, MsWorkspace* w, hipStream_t s) {
    k_ms_clear<<<dense_grid(g, g->n), 256, 0, s>>>(w->vis, w->fr[0], w->fr[1], g->n);
    BFS_HIP(hipGetLastError());
    BFS_HIP(hipMemsetAsync(w->ctrl, 0, sizeof(MsCtrl), s));
}

void ms_join(bfs_graph* g, MsWorkspace* w, const int32_t* slots, const int32_t* roots, int32_t count, int lvl,
             hipStream_t s, int32_t* pinned_stage) {
    if (count <= 0) return;
    if (count > 64) fail(BFS_E_INTERNAL, "at most 64 slots join at once");
    for (int i = 0; i < count; ++i) {
        if (slots[i] < 0 || slots[i] >= 64) fail(BFS_E_INTERNAL, "slot out of range");
        if (roots[i] < 0 || roots[i] >= g->n) fail(BFS_E_ROOT_RANGE, "root out of range");
    }
    // Slots and roots travel through the device staging area behind the ctrl,
    // from the caller's pinned buffer (asynchronous) or a local one (then the
    // copy is awaited before returning).
    int32_t* d_stage = reinterpret_cast<int32_t*>(w->ctrl + 1);
    int32_t local[128];
    int32_t* stage = pinned_stage ? pinned_stage : local;
    for (int i = 0; i < count; ++i) {
        stage[i] = slots[i];
        stage[64 + i] = roots[i];
    }
    BFS_HIP(hipMemcpyAsync(d_stage, stage, 128 * sizeof(int32_t), hipMemcpyHostToDevice, s));
    const bfs_tunables t = current_tunables(g);
    MsParams p = make_params(g, t, w, lvl);
    if (g->off32)
        k_ms_seed<int32_t><<<1, 64, 0, s>>>(p, d_stage, d_stage + 64, count, lvl);
    else
        k_ms_seed<int64_t><<<1, 64, 0, s>>>(p, d_stage, d_stage + 64, count, lvl);
    BFS_HIP(hipGetLastError());
    if (!pinned_stage) BFS_HIP(hipStreamSynchronize(s));  // the local buffer must outlive the copy
}

void ms_step_enqueue(bfs_graph* g, const bfs_tunables& t, MsWorkspace* w, int level, hipStream_t s,
                     bool per_slot) {
    enqueue_level_any(g, t, w, level, per_slot, s);
    k_ms_summary<<<1, 64, 0, s>>>(w->ctrl, level + 1);
    BFS_HIP(hipGetLastError());
    // Only the small tail of the control block (per-slot totals, summaries).
    const size_t from = offsetof(MsCtrl, slot_reached);
    BFS_HIP(hipMemcpyAsync(reinterpret_cast<char*>(w->host_ctrl) + from, reinterpret_cast<char*>(w->ctrl) + from,
                           sizeof(MsCtrl) - from, hipMemcpyDeviceToHost, s));
}

void ms_set_slot(MsWorkspace* w, MsCtrl* staging, int slot, int32_t* lv, int32_t* pa, int32_t start,
                 hipStream_t s) {
    if (slot < 0 || slot >= 64) fail(BFS_E_INTERNAL, "slot out of range");
    staging->out_lv[slot] = lv;
    staging->out_pa[slot] = pa;
    staging->start[slot] = start;
    BFS_HIP(hipMemcpyAsync(&w->ctrl->out_lv[slot], &staging->out_lv[slot], sizeof(int32_t*), hipMemcpyHostToDevice, s));
    BFS_HIP(hipMemcpyAsync(&w->ctrl->out_pa[slot], &staging->out_pa[slot], sizeof(int32_t*), hipMemcpyHostToDevice, s));
    BFS_HIP(hipMemcpyAsync(&w->ctrl->start[slot], &staging->start[slot], sizeof(int32_t), hipMemcpyHostToDevice, s));
}

void ms_retire(bfs_graph* g, MsWorkspace* w, unsigned long long keep, hipStream_t s) {
    k_ms_retire<<<dense_grid(g, g->n), 256, 0, s>>>(w->vis, g->n, keep);
    BFS_HIP(hipGetLastError());
}

void ms_run_batch(bfs_graph* g, const bfs_tunables& t, MsWorkspace* w, const int32_t* roots, int32_t count,
                  int32_t* levels, int32_t* parents, int64_t ld, hipStream_t s, hipEvent_t stop) {
    if (count < 1 || count > 64) fail(BFS_E_INTERNAL, "group size must be 1..64");
    if (w->n != g->n) fail(BFS_E_INTERNAL, "workspace size mismatch");
    if (ld < g->n) fail(BFS_E_INTERNAL, "leading dimension too small");
    // Unreached pairs get -1 either from a fill before the batch (2 x 4 bytes
    // per pair, written in full lines) or from a pass after it that writes
    // only those pairs; the pass is cheaper when the previous batch on this
    // workspace left few pairs unreached (ER 2^22: none, so the 2 GiB fill is
    // saved; R-MAT 22: about 40%, mostly isolated vertices, where the
    // scattered writes cost 0.9 ms against 0.38 ms for the fill).
    const bool pre_fill = w->last_unreached > 0.1;
    if (pre_fill) {
        launch_fill_i32(levels, (int64_t)count * ld, -1, s);
        launch_fill_i32(parents, (int64_t)count * ld, -1, s);
    }
    ms_reset(g, w, s);
    // Output rows and start levels of the group's slots.
    MsCtrl* hc = w->host_ctrl;
    for (int i = 0; i < 64; ++i) {
        hc->out_lv[i] = i < count ? levels + (int64_t)i * ld : nullptr;
        hc->out_pa[i] = i < count ? parents + (int64_t)i * ld : nullptr;
        hc->start[i] = 0;
    }
    BFS_HIP(hipMemcpyAsync(&w->ctrl->out_lv, &hc->out_lv, sizeof(hc->out_lv), hipMemcpyHostToDevice, s));
    BFS_HIP(hipMemcpyAsync(&w->ctrl->out_pa, &hc->out_pa, sizeof(hc->out_pa), hipMemcpyHostToDevice, s));
    BFS_HIP(hipMemcpyAsync(&w->ctrl->start, &hc->start, sizeof(hc->start), hipMemcpyHostToDevice, s));
    int32_t slots[64];
    for (int i = 0; i < count; ++i) slots[i] = i;
    ms_join(g, w, slots, roots, count, 0, s, nullptr);
    // The -1 entries of the pairs the batch did not reach, then the stop event.
    // One thread per vertex in the first round (writes of one row coalesce
    // across a wavefront), at most 16 workgroups per CU.
    const int ug = (int)std::max<int64_t>(1, std::min<int64_t>((g->n + 255) / 256, (int64_t)g->cu_count * 16));
    auto finish = [&] {
        if (!pre_fill) {
            k_ms_unreached<<<ug, 256, 0, s>>>(w->vis, levels, parents, ld, count, g->n);
            BFS_HIP(hipGetLastError());
        }
        if (stop) BFS_HIP(hipEventRecord(stop, s));
    };
    auto note = [&] {  // what the next batch on this workspace chooses from
        const double pairs = (double)count * (double)g->n;
        w->last_unreached = pairs > 0 ? 1.0 - (double)hc->total_disc / pairs : 1.0;
    };
    if (t.persistent > 0) {
        // Every level in one launch; then the totals for the caller.
        if (g->off32)
            launch_batch_persistent<int32_t>(g, t, w, s);
        else
            launch_batch_persistent<int64_t>(g, t, w, s);
        k_ms_summary<<<1, 64, 0, s>>>(w->ctrl, 0);
        BFS_HIP(hipGetLastError());
        finish();
        BFS_HIP(hipMemcpyAsync(hc, w->ctrl, sizeof(MsCtrl), hipMemcpyDeviceToHost, s));
        BFS_HIP(hipStreamSynchronize(s));
        if (!hc->done) fail(BFS_E_INTERNAL, "batch ended without an empty frontier");
        note();
        return;
    }
    // Per-level launches, enqueued in chunks; the host reads the done flag
    // between chunks. The first chunk covers the level steps the previous
    // batch on this workspace needed (batches of one graph have similar
    // depths), the step that finds the frontier empty included; when it is
    // expected to end the batch, the final pass and the stop event go in
    // before the host waits. If the batch goes on, a later chunk repeats both
    // (the pass only writes pairs still unreached, which later levels then
    // overwrite).
    const int expect = w->last_levels;
    int lvl = 0;
    int chunk = expect > 0 ? expect : 8;
    bool finished = false;
    while (true) {
        for (int i = 0; i < chunk; ++i) enqueue_level_any(g, t, w, lvl + i, false, s);
        lvl += chunk;
        k_ms_summary<<<1, 64, 0, s>>>(w->ctrl, lvl);
        BFS_HIP(hipGetLastError());
        finished = expect > 0 && lvl >= expect;
        if (finished) finish();
        BFS_HIP(hipMemcpyAsync(hc, w->ctrl, sizeof(MsCtrl), hipMemcpyDeviceToHost, s));
        BFS_HIP(hipStreamSynchronize(s));
        if (hc->done || lvl > g->n + 1) break;
        finished = false;
        chunk = chunk < 64 ? chunk * 2 : 64;
    }
    if (hc->done) {
        w->last_levels = hc->num_levels + 1;
        note();
    }
    if (!finished) {
        finish();
        BFS_HIP(hipStreamSynchronize(s));
    }
}

}  // namespace bfs
