// Single-root level-synchronous top-down BFS for gfx950.
//
// Method (paper section 3.1, Algorithm 1; parallel form section 3.2,
// Algorithm 2; data structures section 3.3.1): the current layer and the
// visited set are bitmaps of 32-bit words (vertex v -> word v>>5, bit v&31, as
// in Listing 1). Every vertex u of the current layer scans Adj[u]; a neighbour
// whose visited bit is clear is marked visited, gets level k+1 and parent u,
// and joins the next layer. Any of several racing discoverers is a valid parent
// (section 3.2).
//
// Bitmap updates (tunable update_mode):
//   1 (default) the paper's atomic-free scheme (section 3.3.2, Algorithm 3):
//     discoverers set the visited bit with a plain read-modify-write, which may
//     lose concurrent updates to the same 32-bit word, and write levels[v] and
//     parents[v], which cannot race at bit level. A restoration pass then
//     rebuilds every touched word exactly from the level array (the paper uses
//     a negative predecessor marker for the same purpose) and derives the next
//     layer's bitmap. On gfx950 device-scope atomics execute far from the
//     compute units (about a tenth of the random-load rate), so this is the
//     faster scheme here too.
//   2 claim with atomicOr on the visited word: its returned old value names
//     exactly one winner; the restoration pass only diffs the bitmaps.
//
// One level = two launches:
//   k_expand   frontier bitmap -> neighbour visits. Each wavefront owns a
//              contiguous run of frontier words; it pops set bits with ballot +
//              mbcnt into an LDS ring (dense batches of 64), reads row bounds,
//              expands rows of degree <= T1 packed across the lanes (prefix sum
//              + binary search) and rows with T1 < d <= T2 one wavefront each.
//              Frontier rows with d > T2 come from a list that the previous
//              restore pass compacted; their concatenated arcs are split evenly
//              over all workgroups (one workgroup per row, several for hubs).
//   k_restore  exact next-layer bits per touched word, visited snapshot,
//              next frontier bitmap, per-level discovered count, and the list
//              of the next frontier's big rows: one segment per restore block,
//              placed with a workgroup prefix sum (no atomics).
// Levels are enqueued in chunks; the host reads a done flag between chunks.
//
// Coherence: the eight XCDs have private L2 caches, so a plain load in one
// launch may return a line that another XCD rewrote in an earlier launch. All
// state that crosses launches (levels, visited snapshot, frontier, counters,
// big-row list) is therefore read with device-scope loads, except the per-arc
// visited probe: it stays a plain load used only as a filter, and a candidate
// it lets through is confirmed on the level array with a device-scope load
// before it is claimed.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bfs_internal.h"

namespace bfs {

namespace {

constexpr int kUnroll = 2;  // arcs per lane in flight per expansion step

struct SingleParams {
    const void* off;
    const int32_t* col;
    int32_t n;
    int32_t root;
    int64_t words;  // padded 32-bit words per bitmap (multiple of 64)
    int32_t* levels;
    int32_t* parents;
    uint32_t* vis;
    uint32_t* vis_prev;
    uint32_t* fr;
    Ctrl* ctrl;
    unsigned long long* arcs_slot;     // per expansion block
    unsigned long long* reached_slot;  // per restore block
    const uint32_t* bigmap;   // rows with degree > T2
    int32_t* bl_u;            // big frontier rows, one segment per restore block
    uint32_t* bl_pre;         // their exclusive arc offsets within the segment
    uint32_t* seg_cnt;        // rows per segment
    uint32_t* seg_arcs;       // arcs per segment
    const int32_t* seg_start; // first list slot of each segment
    int32_t restore_grid;
    int32_t t1;
};

constexpr int kMinBigShare = 1024;  // fewest big-row arcs handed to one workgroup

// Cross-kernel shared state (bitmaps, level array, lists, counters) is read and
// written with device-scope accesses: each XCD has its own L2, and a plain load
// may otherwise hit a line another XCD has since rewritten in an earlier kernel.
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

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const int lo = __shfl_xor((int)(uint32_t)x, d, 64);
        const int hi = __shfl_xor((int)(uint32_t)(x >> 32), d, 64);
        x += ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
    }
    return x;
}

__device__ __forceinline__ int64_t shfl64(int64_t x, int src) {
    int lo = __shfl((int)(uint32_t)(uint64_t)x, src, 64);
    int hi = __shfl((int)(uint32_t)((uint64_t)x >> 32), src, 64);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Exclusive prefix sum over a workgroup of BLOCK threads; returns the total.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t& excl, uint32_t* tmp) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int incl = wave_incl_scan((int)x, lane);
    if (lane == 63) tmp[wid] = (uint32_t)incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / 64; ++i) {
        const uint32_t t = tmp[i];
        if (i < wid) before += t;
        total += t;
    }
    __syncthreads();
    excl = before + (uint32_t)incl - x;
    return total;
}

template <typename OffT>
__device__ __forceinline__ int64_t load_off(const void* off, int64_t i) {
    return (int64_t) static_cast<const OffT*>(off)[i];
}

__device__ __forceinline__ unsigned long long* stripe(Ctrl* c, int parity, int s) {
    return &c->newcnt[parity][s * kStripeStride];
}

// Visit up to U arcs per lane: gather neighbour ids, filter on the visited
// word, then mark (plain read-modify-write or atomicOr) and write level/parent.
template <bool kAtomic, int U>
__device__ __forceinline__ void visit_arcs(const SingleParams& p, const int64_t (&pos)[U], const bool (&ok)[U],
                                           const int32_t (&par)[U], int lvl) {
    int32_t v[U];
#pragma unroll
    for (int i = 0; i < U; ++i) v[i] = ok[i] ? __builtin_nontemporal_load(p.col + pos[i]) : 0;
    uint32_t w[U];
#pragma unroll
    for (int i = 0; i < U; ++i) w[i] = ok[i] ? p.vis[v[i] >> 5] : ~0u;
    if (kAtomic) {
        uint32_t old[U];
        bool need[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint32_t b = 1u << (v[i] & 31);
            need[i] = !(w[i] & b);
            old[i] = b;
            if (need[i]) old[i] = atomicOr(p.vis + (v[i] >> 5), b);
        }
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint32_t b = 1u << (v[i] & 31);
            if (need[i] && !(old[i] & b)) {
                p.levels[v[i]] = lvl;
                p.parents[v[i]] = par[i];
            }
        }
    } else {
        // The plain load above is only a filter: its line may be stale in this
        // XCD's L2. A candidate is confirmed on the level array, which earlier
        // kernels wrote and a device-scope load reads exactly: -1 means not
        // reached in any earlier level.
        int lv_now[U];
#pragma unroll
        for (int i = 0; i < U; ++i) lv_now[i] = (!(w[i] & (1u << (v[i] & 31)))) ? ld(p.levels + v[i]) : 0;
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint32_t b = 1u << (v[i] & 31);
            if (!(w[i] & b) && lv_now[i] == -1) {
                p.vis[v[i] >> 5] = w[i] | b;  // may lose a concurrent update: restored later
                p.levels[v[i]] = lvl;
                p.parents[v[i]] = par[i];
            }
        }
    }
}

template <bool kAtomic, int U>
__device__ __forceinline__ void expand_row(const SingleParams& p, int64_t beg, int64_t d, int32_t u, int t,
                                           int nthreads, int lvl) {
    for (int64_t j0 = 0; j0 < d; j0 += (int64_t)nthreads * U) {
        int64_t pos[U];
        bool ok[U];
        int32_t par[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const int64_t j = j0 + (int64_t)i * nthreads + t;
            ok[i] = j < d;
            pos[i] = beg + j;
            par[i] = u;
        }
        visit_arcs<kAtomic, U>(p, pos, ok, par, lvl);
    }
}

// One batch of up to 64 staged frontier vertices (valid lanes only). Rows of
// degree <= T1 are expanded packed: arc a of the batch belongs to the entry e
// with excl[e] <= a < incl[e]. Larger rows get the whole wavefront each.
template <typename OffT, bool kAtomic>
__device__ __forceinline__ void process_batch(const SingleParams& p, int32_t u, bool valid, int lane, int lvl,
                                              unsigned long long& arcs) {
    int64_t beg = 0, d = 0;
    if (valid) {
        beg = load_off<OffT>(p.off, u);
        d = load_off<OffT>(p.off, (int64_t)u + 1) - beg;
    }
    arcs += (unsigned long long)d;
    const bool small = valid && d <= p.t1;
    const int ds = small ? (int)d : 0;
    const int incl = wave_incl_scan(ds, lane);
    const int excl = incl - ds;
    const int total = __shfl(incl, 63, 64);
    for (int base = 0; base < total; base += 64 * kUnroll) {
        int64_t pos[kUnroll];
        bool ok[kUnroll];
        int32_t par[kUnroll];
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
            const int64_t b = shfl64(beg, lo);
            par[i] = __shfl(u, lo, 64);
            pos[i] = b + (ac - ex);
        }
        visit_arcs<kAtomic, kUnroll>(p, pos, ok, par, lvl);
    }
    uint64_t mm = __ballot(valid && !small && d > 0);
    while (mm) {
        const int e = __builtin_ctzll(mm);
        mm &= mm - 1;
        expand_row<kAtomic, kUnroll>(p, shfl64(beg, e), shfl64(d, e), __shfl(u, e, 64), lane, 64, lvl);
    }
}

constexpr int kMaxRestoreGrid = 2048;

template <int BLOCK>
struct ExpandShared {
    static constexpr int NW = BLOCK / 64;
    uint32_t ring[NW][128];
    uint32_t segpre[kMaxRestoreGrid + 1];  // exclusive prefix of segment arcs
    uint32_t tmp[BLOCK / 64];
    unsigned long long red[NW];
    unsigned long long found;
    unsigned long long big_total;
    int64_t row_beg;   // broadcast of the big row being expanded
    int64_t row_len;
    int32_t row_u;
};

// a0: levels/parents = -1, bitmaps cleared, root seeded, counters reset.
template <typename OffT, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_init(SingleParams p, int nslots) {
    const int64_t gtid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t gsize = (int64_t)gridDim.x * BLOCK;
    const int64_t n4 = p.n / 4;
    const bool aligned = ((reinterpret_cast<uintptr_t>(p.levels) | reinterpret_cast<uintptr_t>(p.parents)) & 15) == 0;
    if (aligned) {
        int4* lv4 = reinterpret_cast<int4*>(p.levels);
        int4* pa4 = reinterpret_cast<int4*>(p.parents);
        for (int64_t i = gtid; i < n4; i += gsize) {
            int4 a = make_int4(-1, -1, -1, -1), b = make_int4(-1, -1, -1, -1);
            if ((p.root >> 2) == i) {
                const int k = p.root & 3;
                if (k == 0) { a.x = 0; b.x = p.root; }
                if (k == 1) { a.y = 0; b.y = p.root; }
                if (k == 2) { a.z = 0; b.z = p.root; }
                if (k == 3) { a.w = 0; b.w = p.root; }
            }
            lv4[i] = a;
            pa4[i] = b;
        }
    }
    for (int64_t i = (aligned ? n4 * 4 : 0) + gtid; i < p.n; i += gsize) {
        p.levels[i] = (i == p.root) ? 0 : -1;
        p.parents[i] = (i == p.root) ? p.root : -1;
    }
    const int64_t rw = p.root >> 5;
    const uint32_t rb = 1u << (p.root & 31);
    for (int64_t w = gtid; w < p.words; w += gsize) {
        const uint32_t x = (w == rw) ? rb : 0u;
        p.vis[w] = x;
        p.vis_prev[w] = x;
        p.fr[w] = x;
    }
    for (int64_t i = gtid; i < nslots; i += gsize) {
        p.arcs_slot[i] = 0;
        p.reached_slot[i] = 0;
    }
    // The root is the whole first frontier; when its row is big it is the only
    // entry of the big-row list (in the segment of its restore block).
    const bool root_big = (p.bigmap[rw] >> (p.root & 31)) & 1u;
    const int root_seg = (int)((rw / kRestoreBlock) % p.restore_grid);
    const int64_t root_deg = load_off<OffT>(p.off, (int64_t)p.root + 1) - load_off<OffT>(p.off, p.root);
    for (int64_t i = gtid; i < p.restore_grid; i += gsize) {
        const bool here = root_big && i == root_seg;
        p.seg_cnt[i] = here ? 1u : 0u;
        p.seg_arcs[i] = here ? (uint32_t)root_deg : 0u;
        if (here) {
            p.bl_u[p.seg_start[i]] = p.root;
            p.bl_pre[p.seg_start[i]] = 0;
        }
    }
    for (int64_t i = gtid; i < 2 * kStripes; i += gsize) {
        *stripe(p.ctrl, (int)(i / kStripes), (int)(i % kStripes)) = (i == 0) ? 1ull : 0ull;
        p.ctrl->bigarcs[i / kStripes][(i % kStripes) * kStripeStride] = (i == 0 && root_big) ? (unsigned long long)root_deg : 0ull;
    }
    if (gtid == 0) {
        p.ctrl->done = 0;
        p.ctrl->num_levels = 0;
        p.ctrl->reached = 0;
        p.ctrl->arcs = 0;
    }
}

// Expansion of level `lvl` (frontier bitmap p.fr).
template <typename OffT, int BLOCK, bool kAtomic>
__global__ __launch_bounds__(BLOCK) void k_expand(SingleParams p, int lvl) {
    constexpr int NW = BLOCK / 64;
    __shared__ ExpandShared<BLOCK> sh;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t G = gridDim.x, bid = blockIdx.x;
    if (ld(&p.ctrl->done)) return;

    // Termination: the restore pass of the previous level counted this frontier.
    if (tid < 64) {
        unsigned long long c = ld(stripe(p.ctrl, lvl & 1, tid));
        c = wave_sum(c);
        if (tid == 0) sh.found = c;
        if (bid == 0) st(stripe(p.ctrl, (lvl + 1) & 1, tid), 0ull);  // counters for the next level
    }
    __syncthreads();
    if (sh.found == 0) {
        if (bid == 0 && tid == 0) {
            p.ctrl->num_levels = lvl;
            __hip_atomic_store(&p.ctrl->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    unsigned long long arcs = 0;

    // ---- rows of degree > T2: the level's big-row arcs, split evenly
    if (tid < 64) {
        unsigned long long c = ld(&p.ctrl->bigarcs[lvl & 1][tid * kStripeStride]);
        c = wave_sum(c);
        if (tid == 0) sh.big_total = c;
        if (bid == 0) st(&p.ctrl->bigarcs[(lvl + 1) & 1][tid * kStripeStride], 0ull);
    }
    __syncthreads();
    const int64_t ta = (int64_t)sh.big_total;
    if (ta > 0) {
        int64_t per = (ta + G - 1) / G;
        if (per < kMinBigShare) per = kMinBigShare;
        const int64_t a0 = bid * per;
        const int64_t a1 = a0 + per < ta ? a0 + per : ta;
        if (a0 < a1) {
            // Exclusive prefix of the segment totals (one segment per restore block).
            const int R = p.restore_grid;
            constexpr int PER_T = (kMaxRestoreGrid + BLOCK - 1) / BLOCK;
            uint32_t vals[PER_T];
            uint32_t mine = 0;
#pragma unroll
            for (int k = 0; k < PER_T; ++k) {
                const int i = tid * PER_T + k;
                vals[k] = i < R ? ld(p.seg_arcs + i) : 0u;
                mine += vals[k];
            }
            uint32_t excl;
            block_excl_scan<BLOCK>(mine, excl, sh.tmp);
#pragma unroll
            for (int k = 0; k < PER_T; ++k) {
                const int i = tid * PER_T + k;
                if (i <= R) sh.segpre[i] = excl;
                excl += vals[k];
            }
            __syncthreads();
            // Walk the rows covering [a0, a1): thread 0 locates each piece, the
            // whole workgroup expands it.
            int seg = 0, idx = 0;
            if (tid == 0) {
                int lo = 0, hi = R - 1;  // last segment with segpre <= a0
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if ((int64_t)sh.segpre[mid] <= a0)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                while (lo < R - 1 && (int64_t)sh.segpre[lo + 1] <= a0) ++lo;
                seg = lo;
                const int64_t local = a0 - (int64_t)sh.segpre[seg];
                const int first = p.seg_start[seg];
                int l2 = 0, h2 = (int)ld(p.seg_cnt + seg) - 1;  // last row with offset <= local
                while (l2 < h2) {
                    const int mid = (l2 + h2 + 1) >> 1;
                    if ((int64_t)ld(p.bl_pre + first + mid) <= local)
                        l2 = mid;
                    else
                        h2 = mid - 1;
                }
                idx = l2;
            }
            int64_t pos = a0;
            while (pos < a1) {
                if (tid == 0) {
                    while (seg < R && idx >= (int)ld(p.seg_cnt + seg)) {  // next non-empty segment
                        ++seg;
                        idx = 0;
                    }
                }
                if (tid == 0 && seg >= R) sh.row_len = 0;  // list exhausted (cannot happen: a1 <= total)
                if (tid == 0 && seg < R) {
                    const int slot = p.seg_start[seg] + idx;
                    const int32_t u = ld(p.bl_u + slot);
                    const int64_t row_start = (int64_t)sh.segpre[seg] + ld(p.bl_pre + slot);
                    const int64_t beg = load_off<OffT>(p.off, u);
                    const int64_t deg = load_off<OffT>(p.off, (int64_t)u + 1) - beg;
                    const int64_t end = row_start + deg < a1 ? row_start + deg : a1;
                    sh.row_u = u;
                    sh.row_beg = beg + (pos - row_start);
                    sh.row_len = end - pos;
                    ++idx;
                }
                __syncthreads();
                const int64_t len = sh.row_len;
                if (len <= 0) break;
                expand_row<kAtomic, kUnroll>(p, sh.row_beg, len, sh.row_u, tid, BLOCK, lvl + 1);
                if (tid == 0) arcs += (unsigned long long)len;
                pos += len;
                __syncthreads();
            }
        }
    }

    // ---- every other frontier vertex: a contiguous run of words per wavefront
    const int64_t waves = G * NW;
    const int64_t gw = bid * NW + wid;
    const int64_t wpw = (p.words + waves - 1) / waves;
    const int64_t w0 = gw * wpw;
    const int64_t w1 = w0 + wpw < p.words ? w0 + wpw : p.words;
    uint32_t head = 0, tail = 0;
    for (int64_t base = w0; base < w1; base += 64) {
        const int64_t wi = base + lane;
        uint32_t word = wi < w1 ? (ld(p.fr + wi) & ~p.bigmap[wi]) : 0u;
        while (true) {
            const bool has = word != 0;
            const uint64_t m = __ballot(has);
            if (m == 0) break;
            if (has) {
                const int bit = __builtin_ctz(word);
                word &= word - 1;
                sh.ring[wid][(tail + rank_in(m)) & 127] = (uint32_t)(wi * 32 + bit);
            }
            tail += __popcll(m);
            if (tail - head >= 64) {
                const int32_t u = (int32_t)sh.ring[wid][(head + lane) & 127];
                head += 64;
                process_batch<OffT, kAtomic>(p, u, true, lane, lvl + 1, arcs);
            }
        }
    }
    if (tail != head) {
        const int cnt = (int)(tail - head);
        const bool valid = lane < cnt;
        const int32_t u = valid ? (int32_t)sh.ring[wid][(head + lane) & 127] : 0;
        process_batch<OffT, kAtomic>(p, u, valid, lane, lvl + 1, arcs);
    }

    // ---- block total of scanned arcs (plain update of this block's own slot)
    const unsigned long long asum = wave_sum(arcs);
    if (lane == 0) sh.red[wid] = asum;
    __syncthreads();
    if (tid == 0) {
        unsigned long long a = 0;
        for (int i = 0; i < NW; ++i) a += sh.red[i];
        p.arcs_slot[bid] += a;
    }
}

// Restoration of level `lvl`: exact new bits per touched word, visited snapshot,
// next frontier bitmap, the discovered count (striped), and the compacted list
// of the next frontier's rows above T2 (this block's segment).
template <typename OffT, bool kAtomic>
__global__ __launch_bounds__(kRestoreBlock) void k_restore(SingleParams p, int lvl) {
    constexpr int BLOCK = kRestoreBlock;
    __shared__ unsigned long long red[BLOCK / 64];
    __shared__ uint32_t tmp[BLOCK / 64];
    if (ld(&p.ctrl->done)) return;
    const int tid = threadIdx.x;
    const int64_t G = gridDim.x, bid = blockIdx.x;
    const int next = lvl + 1;
    unsigned long long found = 0;
    uint32_t seg_n = 0, seg_a = 0;  // running totals of this block's segment
    const int32_t first = p.seg_start[bid];
    for (int64_t c = bid; c * BLOCK < p.words; c += G) {
        const int64_t w = c * BLOCK + tid;
        const int lane = tid & 63;
        uint32_t cur = 0, prev = 0, exact = 0;
        if (w < p.words) {
            cur = ld(p.vis + w);
            prev = ld(p.vis_prev + w);
        }
        const bool touched = w < p.words && cur != prev;
        if (kAtomic) {
            exact = touched ? (cur & ~prev) : 0u;
        } else {
            // A racing read-modify-write may have dropped bits (of this level,
            // or of earlier ones through a stale filter read; the snapshot
            // puts those back), never added foreign ones, and always leaves
            // one of its bits set: the level array says exactly who was
            // discovered. Two touched words per step: each half-wave reads
            // one word's 32 levels.
            uint64_t tm = __ballot(touched);
            const int64_t wave_w0 = c * BLOCK + (tid & ~63);
            while (tm) {
                const int wa = __builtin_ctzll(tm);
                tm &= tm - 1;
                int wb = -1;
                if (tm) {
                    wb = __builtin_ctzll(tm);
                    tm &= tm - 1;
                }
                const int src = lane < 32 ? wa : wb;
                const int64_t v = (wave_w0 + src) * 32 + (lane & 31);
                const bool okl = src >= 0 && v < p.n;
                const int lvv = okl ? ld(p.levels + v) : -1;
                const uint64_t m = __ballot(lvv == next);
                if (lane == wa) exact = (uint32_t)m;
                if (lane == wb) exact = (uint32_t)(m >> 32);
            }
        }
        if (touched) {
            const uint32_t nv = prev | exact;
            if (cur != nv) st(p.vis + w, nv);
            st(p.vis_prev + w, nv);
        }
        if (w < p.words) {
            st(p.fr + w, exact);
            found += (unsigned long long)__popc(exact);
        }
        // Append the next frontier's big rows of this chunk to the segment.
        const uint32_t big = w < p.words ? (exact & p.bigmap[w]) : 0u;
        uint32_t my_arcs = 0;
        for (uint32_t x = big; x; x &= x - 1) {
            const int64_t u = w * 32 + __builtin_ctz(x);
            my_arcs += (uint32_t)(load_off<OffT>(p.off, u + 1) - load_off<OffT>(p.off, u));
        }
        uint32_t cnt_excl, arc_excl;
        const uint32_t cnt_tot = block_excl_scan<BLOCK>((uint32_t)__popc(big), cnt_excl, tmp);
        const uint32_t arc_tot = block_excl_scan<BLOCK>(my_arcs, arc_excl, tmp);
        if (big) {
            uint32_t slot = first + seg_n + cnt_excl;
            uint32_t at = seg_a + arc_excl;
            for (uint32_t x = big; x; x &= x - 1) {
                const int64_t u = w * 32 + __builtin_ctz(x);
                st(p.bl_u + slot, (int32_t)u);
                st(p.bl_pre + slot, at);
                at += (uint32_t)(load_off<OffT>(p.off, u + 1) - load_off<OffT>(p.off, u));
                ++slot;
            }
        }
        seg_n += cnt_tot;
        seg_a += arc_tot;
    }
    found = wave_sum(found);
    if ((tid & 63) == 0) red[tid >> 6] = found;
    __syncthreads();
    if (tid == 0) {
        unsigned long long a = 0;
        for (int i = 0; i < BLOCK / 64; ++i) a += red[i];
        if (a) {
            atomicAdd(stripe(p.ctrl, next & 1, (int)(bid % kStripes)), a);
            p.reached_slot[bid] += a;
        }
        st(p.seg_cnt + bid, seg_n);
        st(p.seg_arcs + bid, seg_a);
        if (seg_a) atomicAdd(&p.ctrl->bigarcs[next & 1][(bid % kStripes) * kStripeStride], (unsigned long long)seg_a);
    }
}

__global__ void k_stats(Ctrl* c, const unsigned long long* arcs_slot, const unsigned long long* reached_slot,
                        int nslots) {
    __shared__ unsigned long long ra[256], rr[256];
    unsigned long long a = 0, r = 0;
    for (int i = threadIdx.x; i < nslots; i += 256) {
        a += arcs_slot[i];
        r += reached_slot[i];
    }
    ra[threadIdx.x] = a;
    rr[threadIdx.x] = r;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            ra[threadIdx.x] += ra[threadIdx.x + s];
            rr[threadIdx.x] += rr[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        c->arcs = ra[0];
        c->reached = rr[0] + 1;
    }
}

template <typename OffT>
__global__ void k_validate_csr(const OffT* off, const int32_t* col, int64_t n, int64_t nnz, int* err) {
    const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        if (off[0] != 0) atomicOr(err, 1);
        if ((int64_t)off[n] != nnz) atomicOr(err, 2);
    }
    for (int64_t v = t; v < n; v += gsize)
        if (off[v + 1] < off[v]) atomicOr(err, 4);
    for (int64_t j = t; j < nnz; j += gsize)
        if (col[j] < 0 || col[j] >= n) atomicOr(err, 8);
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t value) {
    const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gsize) p[i] = value;
}

template <typename K>
int occupancy_of(K kernel, int block) {
    int occ = 0;
    hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, block, 0), "occupancy query");
    return occ;
}

struct Grids {
    int expand;
    int restore;
};

template <typename OffT, int BLOCK, bool kAtomic>
Grids grids_for(bfs_graph* g, const bfs_tunables& t, int64_t nslots) {
    static const int occ = occupancy_of(k_expand<OffT, BLOCK, kAtomic>, BLOCK);
    const int bpc = t.blocks_per_cu > 0 && (occ < 1 || t.blocks_per_cu < occ) ? t.blocks_per_cu : (occ > 0 ? occ : 1);
    int64_t ge = (int64_t)bpc * g->cu_count;
    ge = std::max<int64_t>(1, std::min(ge, nslots));
    if (g->restore_grid < 1 || g->restore_grid > kMaxRestoreGrid || g->restore_grid > nslots)
        fail(BFS_E_INTERNAL, "restore grid out of range");
    return Grids{(int)ge, g->restore_grid};
}

template <typename OffT, int BLOCK, bool kAtomic>
void launch_typed(bfs_graph* g, const bfs_tunables& t, Workspace* w, SingleParams& p, hipStream_t s) {
    const Grids gr = grids_for<OffT, BLOCK, kAtomic>(g, t, w->nslots);
    const int init_grid = (int)std::min<int64_t>(std::max<int64_t>(p.n / 4, p.words) / BLOCK + 1, 4096);
    k_init<OffT, BLOCK><<<init_grid, BLOCK, 0, s>>>(p, (int)w->nslots);
    BFS_HIP(hipGetLastError());
    // Levels are enqueued in chunks; between chunks the host reads the done flag.
    int lvl = 0;
    int chunk = 8;
    while (true) {
        for (int i = 0; i < chunk; ++i) {
            k_expand<OffT, BLOCK, kAtomic><<<gr.expand, BLOCK, 0, s>>>(p, lvl + i);
            k_restore<OffT, kAtomic><<<gr.restore, kRestoreBlock, 0, s>>>(p, lvl + i);
        }
        BFS_HIP(hipGetLastError());
        lvl += chunk;
        BFS_HIP(hipMemcpyAsync(&w->host_ctrl->done, &p.ctrl->done, sizeof(int), hipMemcpyDeviceToHost, s));
        BFS_HIP(hipStreamSynchronize(s));
        if (w->host_ctrl->done || lvl > p.n + 1) break;
        chunk = chunk < 64 ? chunk * 2 : 64;
    }
}

}  // namespace

void launch_single(bfs_graph* g, const bfs_tunables& t, Workspace* w, int32_t root, int32_t* levels,
                   int32_t* parents, hipStream_t s) {
    // Host-side checks of what the kernels assume about their buffers.
    if (root < 0 || root >= g->n) fail(BFS_E_ROOT_RANGE, "root out of range");
    if (w->words * 32 < g->n || w->words % 64 != 0) fail(BFS_E_INTERNAL, "workspace bitmaps too small");
    if (!levels || !parents) fail(BFS_E_INVALID_ARG, "NULL output");
    if (g->big_threshold != t.wave_max_degree) fail(BFS_E_INTERNAL, "big-row table out of date");
    SingleParams p{};
    p.off = g->d_off;
    p.col = g->d_col;
    p.n = (int32_t)g->n;
    p.root = root;
    p.words = w->words;
    p.levels = levels;
    p.parents = parents;
    p.vis = w->vis;
    p.vis_prev = w->vis_prev;
    p.fr = w->fr;
    p.ctrl = w->ctrl;
    p.arcs_slot = w->slots;
    p.reached_slot = w->slots + w->nslots;
    p.bigmap = g->d_bigmap;
    p.bl_u = w->bl_u;
    p.bl_pre = w->bl_pre;
    p.seg_cnt = w->seg_cnt;
    p.seg_arcs = w->seg_arcs;
    p.seg_start = g->d_seg_start;
    p.restore_grid = g->restore_grid;
    p.t1 = t.small_max_degree;
    if (w->big_capacity < g->num_big) fail(BFS_E_INTERNAL, "big-row list too small");
    const bool atomic = t.update_mode == 2;
#define BFS_LAUNCH(OFFT, BS)                                         \
    do {                                                             \
        if (atomic)                                                  \
            launch_typed<OFFT, BS, true>(g, t, w, p, s);             \
        else                                                         \
            launch_typed<OFFT, BS, false>(g, t, w, p, s);            \
    } while (0)
    if (g->off32) {
        if (t.block_size == 512)
            BFS_LAUNCH(int32_t, 512);
        else
            BFS_LAUNCH(int32_t, 256);
    } else {
        if (t.block_size == 512)
            BFS_LAUNCH(int64_t, 512);
        else
            BFS_LAUNCH(int64_t, 256);
    }
#undef BFS_LAUNCH
}

void launch_single_stats(Workspace* w, hipStream_t s) {
    k_stats<<<1, 256, 0, s>>>(w->ctrl, w->slots, w->slots + w->nslots, (int)w->nslots);
    BFS_HIP(hipGetLastError());
}

void validate_device_csr(const void* off, bool off32, const int32_t* col, int64_t n, int64_t nnz) {
    int* d_err = nullptr;
    BFS_HIP(hipMalloc(&d_err, sizeof(int)));
    int err = 0;
    try {
        BFS_HIP(hipMemset(d_err, 0, sizeof(int)));
        const int64_t work = n > nnz ? n : nnz;
        const int blocks = (int)(work / 256 + 1 < 8192 ? work / 256 + 1 : 8192);
        if (off32)
            k_validate_csr<int32_t><<<blocks, 256>>>(static_cast<const int32_t*>(off), col, n, nnz, d_err);
        else
            k_validate_csr<int64_t><<<blocks, 256>>>(static_cast<const int64_t*>(off), col, n, nnz, d_err);
        BFS_HIP(hipGetLastError());
        BFS_HIP(hipMemcpy(&err, d_err, sizeof(int), hipMemcpyDeviceToHost));
    } catch (...) {
        (void)hipFree(d_err);
        throw;
    }
    (void)hipFree(d_err);
    if (err) fail(BFS_E_INVALID_GRAPH, "device CSR failed validation (code " + std::to_string(err) + ")");
}

void launch_fill_i32(int32_t* ptr, int64_t count, int32_t value, hipStream_t s) {
    if (count <= 0) return;
    const int blocks = (int)(count / 1024 + 1 < 4096 ? count / 1024 + 1 : 4096);
    k_fill_i32<<<blocks, 256, 0, s>>>(ptr, count, value);
    BFS_HIP(hipGetLastError());
}

}  // namespace bfs
