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
// A small frontier (tunable sparse_frontier) is expanded by k_expand's first
// workgroup alone, which goes on through the small levels after it in the
// same launch (small_levels). Levels are enqueued in chunks; the host reads a
// done flag between chunks.
//
// Coherence: the eight XCDs have private L2 caches. Launch boundaries make
// them agree (a plain load sees what another XCD wrote in an earlier launch),
// but within a launch an XCD's L2 does not see other XCDs' stores. Shared state
// is read and written with device-scope accesses; the per-arc visited probe is
// a plain load used only as a filter, and a candidate it lets through is
// confirmed on the level array with a device-scope load, which sees claims that
// other XCDs made earlier in the same launch, before it is claimed.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bfs_internal.h"

namespace bfs {

namespace {

constexpr int kUnroll = 2;     // arcs per lane in flight: one wavefront per row (T1 < d <= T2)
constexpr int kLbsUnroll = 8;  // arcs per lane in flight: packed rows (d <= T1)
constexpr int kBigUnroll = 8;  // arcs per lane in flight: rows above T2
// What a walk over staged big-row arcs does with each arc.
constexpr int kWalkProbe = 0;    // probe, confirm and claim (visit_arcs)
constexpr int kWalkBlocked = 1;  // heads in the LDS block slice (visit_blocked)
constexpr int kWalkBinned = 2;   // to the destination bins (visit_binned)
constexpr int kBuFirst = 4;       // bottom-up: arcs each lane checks before its wavefront helps
constexpr int kRebuildPairs = 8;   // restore: pairs of touched words whose levels are read per round
// Big-row arcs per expansion workgroup above which a level with a small
// frontier (a hub level) still takes the LDS copy of the visited bits: the
// copy filters repeat heads within the workgroup (R-MAT 24: -1.2% per BFS,
// -5% on roots with the largest hub levels; R-MAT 26 -1.9%; R-MAT 20 no change).
constexpr int64_t kHubLdsArcs = 4096;

struct SingleParams {
    const void* off;
    const int32_t* col;
    int32_t n;
    int32_t root;
    int64_t words;  // padded 32-bit words per bitmap (multiple of 64)
    // Levels by the run's vertex ids (read by restore and claims): the caller's
    // level array, or on the degree-ordered copy the level half of an
    // interleaved {level, parent} record per run id.
    int32_t* lv;
    int32_t* out_lv;           // the caller's levels and parents, by caller ids
    int32_t* out_pa;
    const int32_t* new2old;    // run id -> caller id on the degree-ordered copy, else nullptr
    const int32_t* old2new;    // caller id -> run id on the degree-ordered copy, else nullptr
    int32_t root_out;          // the root as a caller id
    uint32_t* vis;
    uint32_t* vis_prev;
    uint32_t* fr;
    Ctrl* ctrl;
    unsigned long long* arcs_slot;     // per expansion block
    unsigned long long* reached_slot;  // per restore block
    const uint32_t* bigmap;   // rows with degree > T2
    const uint32_t* nzmap;    // rows with degree > 0
    int32_t* bl_u;            // big frontier rows, one segment per restore block
    uint32_t* bl_pre;         // their exclusive arc offsets within the segment
    uint32_t* seg_cnt;        // rows per segment
    uint32_t* seg_arcs;       // arcs per segment
    const int32_t* seg_start; // first list slot of each segment
    int32_t restore_grid;
    int32_t t1;
    int32_t min_share;         // fewest big-row arcs handed to one workgroup
    // Rows above T2 grouped by destination block (degree-ordered copy): nblk
    // blocks of 2^blk_shift vertices; bseg holds nblk + 1 local arc offsets per
    // row, by hot rank (nullptr: not grouped). Levels whose big rows have at
    // least blk_min_arcs arcs and whose frontier is large expand them by block.
    // Destination bins of hub levels: bin_e holds {head, parent} entries in a
    // region of bin_k per (bin, expansion workgroup), bin_cnt[workgroup][bin]
    // the entries each region got; a bin is a restore chunk (kRestoreBlock
    // visited words). bin_k 0 = off.
    int2* bin_e;
    uint32_t* bin_cnt;
    int32_t bin_k;
    int32_t bin_groups;        // expansion workgroups (regions per bin)
    int32_t bin_nb;            // bins
    const uint32_t* bseg;
    int32_t bseg_rows;         // rows in bseg
    int32_t nblk;
    int32_t blk_shift;
    int64_t blk_min_arcs;
    // The 32 * hot_words hot vertices sit at bit positions k << hot_shift of
    // the first hot_span visited words (one per word with shift 5, bits 0 and
    // 16 with shift 4). hot_vis is their compact visited bitmap (slot
    // w + k * hot_span for position k of word w), which the restore pass keeps
    // exact and expansion workgroups copy into LDS.
    uint32_t* hot_vis;
    uint32_t* hot_fr;          // compact bitmap of the hot vertices in the frontier (exact per level)
    int32_t hot_words;         // words of hot_vis / hot_fr (0 = off)
    int32_t hot_shift;         // 5 or 4
    int32_t hot_span;          // visited words holding hot vertices: hot_words << hot_shift
    int64_t hot_min_frontier;  // use an LDS copy only for frontiers of at least this many vertices
    // Without the degree-ordered copy: words of the visited bitmap (bottom-up
    // levels: of the frontier bitmap) that workgroups copy whole into LDS (0 = off).
    int32_t full_words;
    int64_t nnz;
    int32_t hybrid;            // levels with large frontiers may run bottom-up (symmetric graphs)
    // Small levels: each restore block lists up to kSmallSeg ids of the next
    // frontier (sl) and counts them (sl_cnt); frontiers of at most s_max
    // vertices and s_arcs arcs are expanded by workgroup 0 alone (s_max 0 = off).
    int32_t* sl;
    int32_t* sl_cnt;
    int32_t s_max;
    int64_t s_arcs;
};


// Shared state (bitmaps, level array, lists, counters) is read and written with
// device-scope accesses. Across launches plain accesses see the same values (a
// probe that rewrote a buffer from one XCD and read it from another in the
// next launch found no stale line), but within a launch each XCD has its own
// L2: a device-scope load of the level array sees the claims other XCDs made
// earlier in the same launch, which keeps duplicate claims down. With plain
// loads throughout, a BFS of R-MAT scale 24 took 8% longer.
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
// Caller id of run id u.
__device__ __forceinline__ int32_t out_id(const SingleParams& p, int32_t u) { return p.new2old ? p.new2old[u] : u; }

// Index of run id v's level in p.lv.
__device__ __forceinline__ int64_t lv_at(const SingleParams& p, int64_t v) { return p.new2old ? 2 * v : v; }

// Discovery of run id v at level lvl from the caller-id parent par. On the
// degree-ordered copy this is one 8-byte record at the run id; the caller's
// arrays are filled by one pass in run order after the last level (cold ids
// keep the caller's order, so that pass writes nearly coalesced).
__device__ __forceinline__ void record(const SingleParams& p, int32_t v, int lvl, int32_t par) {
    if (p.new2old) {
        *reinterpret_cast<int2*>(p.lv + 2 * (int64_t)v) = make_int2(lvl, par);
    } else {
        p.lv[v] = lvl;
        p.out_pa[v] = par;
    }
}

// The same discovery written with device-scope stores, for a pass that reads
// the level array back with device-scope loads in the same launch.
__device__ __forceinline__ void record_st(const SingleParams& p, int32_t v, int lvl, int32_t par) {
    if (p.new2old) {
        st(reinterpret_cast<unsigned long long*>(p.lv + 2 * (int64_t)v),
           ((unsigned long long)(uint32_t)par << 32) | (uint32_t)lvl);
    } else {
        st(p.lv + v, lvl);
        st(p.out_pa + v, par);
    }
}

// Bins are restore chunks: kRestoreBlock visited words of 32 vertices.
static_assert(kRestoreBlock == 256, "a bin is 256 visited words (8192 vertices)");
constexpr int kBinShift = 13;

// Compact-bitmap slot of v if v is hot: position k = (v & 31) >> shift of
// visited word w = v >> 5 < span has slot w + k * span.
__device__ __forceinline__ bool hot_slot(uint32_t v, uint32_t span, uint32_t shift, uint32_t& slot) {
    const uint32_t w = v >> 5;
    slot = w + ((v & 31u) >> shift) * span;
    return (v & ((1u << shift) - 1u)) == 0 && w < span;
}

// A workgroup's LDS copy of visited bits, taken at the start of a level (so a
// set bit is final): either the compact bits of the hot ids, or the first
// words of the visited bitmap itself (bit v). One form covers both, so a
// lookup needs no branch: v is held if v & mask == 0 and its word w = v >> 5
// is below lim, at bit (w << wshift) + ((v & 31) >> shift) * kmul.
//   hot bits:  mask 2^hot_shift - 1, lim hot_span, shift hot_shift, wshift 0, kmul hot_span;
//   whole words: mask 0, lim full_words, shift 0, wshift 5, kmul 1;
//   no copy: lim 0.
struct LdsVis {
    uint32_t* bits;
    uint32_t lim;
    uint32_t mask;
    uint32_t shift;
    uint32_t wshift;
    uint32_t kmul;

    __device__ static LdsVis none(uint32_t* b) { return LdsVis{b, 0u, 0u, 0u, 0u, 0u}; }
    __device__ void set_hot(uint32_t span, uint32_t hshift) {
        lim = span;
        mask = (1u << hshift) - 1u;
        shift = hshift;
        wshift = 0u;
        kmul = span;
    }
    __device__ void set_words(uint32_t words) {
        lim = words;
        mask = 0u;
        shift = 0u;
        wshift = 5u;
        kmul = 1u;
    }
};

// Bit of vertex v in the LDS copy, if the copy holds it.
__device__ __forceinline__ bool lds_slot(const LdsVis& l, int32_t v, uint32_t& bit) {
    const uint32_t u = (uint32_t)v, w = u >> 5;
    bit = (w << l.wshift) + __umul24((u & 31u) >> l.shift, l.kmul);  // both factors below 2^24
    return ((u & l.mask) == 0u) & (w < l.lim);
}

// Hot ids are first looked up in the workgroup's LDS
// copy of the compact hot bitmap (taken at the start of the level, so a set bit
// is final); only the rest, and hot ids not yet visited, probe the global bitmap.
template <bool kAtomic, int U>
__device__ __forceinline__ void visit_arcs(const SingleParams& p, const int64_t (&pos)[U], const bool (&ok)[U],
                                           const int32_t (&par)[U], int lvl, const LdsVis& lds) {
    // Loads are issued by every lane, so no lane mask is set up around them:
    // callers hand idle lanes a valid position (a repeat of a real arc), and
    // lanes with nothing to probe read one shared dummy word (one request per
    // wavefront instruction) and discard it.
    int32_t v[U];
#pragma unroll
    for (int i = 0; i < U; ++i) v[i] = __builtin_nontemporal_load(p.col + pos[i]);
    uint32_t w[U];
    bool in_lds[U];
    uint32_t slot[U], lw[U];
#pragma unroll
    for (int i = 0; i < U; ++i) in_lds[i] = ok[i] & lds_slot(lds, v[i], slot[i]);
    if (lds.lim != 0) {  // the same for the whole workgroup
#pragma unroll
        for (int i = 0; i < U; ++i) lw[i] = lds.bits[in_lds[i] ? slot[i] >> 5 : 0];
    } else {
#pragma unroll
        for (int i = 0; i < U; ++i) lw[i] = 0u;
    }
#pragma unroll
    for (int i = 0; i < U; ++i) {
        const bool known = in_lds[i] & (((lw[i] >> (slot[i] & 31)) & 1u) != 0u);
        const bool need = ok[i] & !known;
        const uint32_t x = p.vis[need ? (uint32_t)v[i] >> 5 : 0u];
        w[i] = need ? x : ~0u;
    }
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
            if (need[i] && !(old[i] & b)) record(p, v[i], lvl, par[i]);
            if (need[i] && in_lds[i]) atomicOr(lds.bits + (slot[i] >> 5), 1u << (slot[i] & 31));
        }
    } else {
        // The plain load above is only a filter: this XCD's L2 line lacks the
        // claims other XCDs made in this launch. A candidate is confirmed on
        // the level array with a device-scope load, which sees them: -1 means
        // not reached yet (a claim racing past it is a duplicate of the same
        // level, which the restoration tolerates).
        int lv_now[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const bool cand = !(w[i] & (1u << (v[i] & 31)));
            const int x = ld(p.lv + (cand ? lv_at(p, v[i]) : 0));
            lv_now[i] = cand ? x : 0;
        }
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint32_t b = 1u << (v[i] & 31);
            if (!(w[i] & b) && lv_now[i] == -1) {
                p.vis[v[i] >> 5] = w[i] | b;  // may lose a concurrent update: restored later
                record(p, v[i], lvl, par[i]);
            }
            if (!(w[i] & b) && in_lds[i]) atomicOr(lds.bits + (slot[i] >> 5), 1u << (slot[i] & 31));  // this workgroup's later probes
        }
    }
}

template <bool kAtomic, int U>
__device__ __forceinline__ void expand_row(const SingleParams& p, int64_t beg, int64_t d, int32_t u, int t,
                                           int nthreads, int lvl, const LdsVis& lds) {
    for (int64_t j0 = 0; j0 < d; j0 += (int64_t)nthreads * U) {
        int64_t pos[U];
        bool ok[U];
        int32_t par[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const int64_t j = j0 + (int64_t)i * nthreads + t;
            ok[i] = j < d;
            pos[i] = beg + (ok[i] ? j : d - 1);  // idle lanes repeat the row's last arc
            par[i] = u;
        }
        visit_arcs<kAtomic, U>(p, pos, ok, par, lvl, lds);
    }
}

// One batch of up to 64 staged frontier vertices (valid lanes only). Rows of
// degree <= T1 are expanded packed: their arcs are numbered consecutively in
// lane order and taken 64 x kLbsUnroll at a time, one arc per lane per window.
// A lane finds the row of its arc from the row starts that fall inside the
// span: each row writes its lane into a per-wavefront byte map at its first
// arc, a ballot over the map gives the window's start positions, and the
// last start at or before the lane names the row (or, with none, the row that
// was open at the end of the previous window). Larger rows get the whole
// wavefront each.
template <typename OffT, bool kAtomic>
__device__ __forceinline__ void process_batch(const SingleParams& p, int32_t u, bool valid, int lane, int lvl,
                                              unsigned long long& arcs, const LdsVis& lds,
                                              uint8_t* starts) {
    constexpr int SPAN = 64 * kLbsUnroll;
    static_assert(SPAN % 256 == 0, "the start map is cleared in 32-bit words, one or more per lane");
    int64_t beg = 0, d = 0;
    int32_t uo = 0;  // the row as a caller id: the parent of its discoveries
    if (valid) {
        beg = load_off<OffT>(p.off, u);
        d = load_off<OffT>(p.off, (int64_t)u + 1) - beg;
        uo = out_id(p, u);
    }
    arcs += (unsigned long long)d;
    const bool small = valid && d <= p.t1;
    const int ds = small ? (int)d : 0;
    const int incl = wave_incl_scan(ds, lane);
    const int excl = incl - ds;
    const int total = __shfl(incl, 63, 64);
    const int64_t rbase = beg - excl;  // column index of packed arc a of this row: rbase + a
    int open = 0;                      // row holding the arc just before the current window
    for (int base = 0; base < total; base += SPAN) {
#pragma unroll
        for (int k = 0; k < SPAN / 256; ++k) reinterpret_cast<uint32_t*>(starts)[k * 64 + lane] = 0xFFFFFFFFu;
        __builtin_amdgcn_wave_barrier();
        if (ds > 0 && excl >= base && excl < base + SPAN) starts[excl - base] = (uint8_t)lane;
        __builtin_amdgcn_wave_barrier();
        int64_t pos[kLbsUnroll];
        bool ok[kLbsUnroll];
        int32_t par[kLbsUnroll];
#pragma unroll
        for (int i = 0; i < kLbsUnroll; ++i) {
            const int here = starts[i * 64 + lane];
            const uint64_t m = __ballot(here != 0xFF) & ((2ull << lane) - 1ull);  // starts at or before this lane
            const int last = m ? 63 - __builtin_clzll(m) : 0;
            const int from_map = __shfl(here, last, 64);
            const int e = m ? from_map : open;
            open = __shfl(e, 63, 64);
            // Lanes past the batch's last arc repeat it (their row is the last one).
            ok[i] = base + i * 64 + lane < total;
            const int ac = ok[i] ? base + i * 64 + lane : total - 1;
            pos[i] = shfl64(rbase, e) + ac;
            par[i] = __shfl(uo, e, 64);
        }
        visit_arcs<kAtomic, kLbsUnroll>(p, pos, ok, par, lvl, lds);
    }
    uint64_t mm = __ballot(valid && !small && d > 0);
    while (mm) {
        const int e = __builtin_ctzll(mm);
        mm &= mm - 1;
        expand_row<kAtomic, kUnroll>(p, shfl64(beg, e), shfl64(d, e), __shfl(uo, e, 64), lane, 64, lvl, lds);
    }
}

template <int BLOCK>
struct ExpandShared {
    static constexpr int NW = BLOCK / 64;
    union {
        struct {
            uint32_t ring[NW][128];    // staged frontier (or unvisited) vertices, one ring per wavefront
            uint32_t bu_bits[NW][64];  // bottom-up: new visited bits of each wavefront's 64-word window
            uint8_t starts[NW][64 * kLbsUnroll];  // packed rows: lane of the row starting at each arc of a span
        } w;
        struct {
            uint32_t segpre[kMaxRestoreGrid + 1];  // exclusive prefix of segment arcs
            uint32_t cntpre[kMaxRestoreGrid + 1];  // exclusive prefix of segment rows
            int64_t start[BLOCK];  // first arc (level-wide numbering, clipped to the share) of a staged row
            int64_t base[BLOCK];   // column index minus arc number for that row
            int32_t u[BLOCK];      // the row's vertex as a caller id
        } big;
    } x;
    uint32_t tmp[BLOCK / 64];
    unsigned long long red[NW];
    unsigned long long found;
    unsigned long long big_total;
    unsigned long long seen;  // hybrid runs: vertices visited before this frontier
    int was_bu;               // hybrid runs: the previous level ran bottom-up
    int done;                 // the run had already ended
    int lvl;                  // the level this step expands
    int shift;                // levels earlier steps ran beyond their own
    int small;                // the frontier is small enough for workgroup 0 alone
    uint32_t s_next;          // small levels: next-frontier entries so far
    int64_t staged_end;  // last arc (exclusive) of the staged big rows
    uint32_t row0;
};

// Prefix sums over the level's big-row list (one segment per restore block):
// arcs (segpre) and rows (cntpre), in LDS. Returns the number of listed rows.
template <int BLOCK>
__device__ __forceinline__ uint32_t big_prefix(const SingleParams& p, ExpandShared<BLOCK>& sh) {
    const int tid = threadIdx.x;
    const int R = p.restore_grid;
    constexpr int PER_T = (kMaxRestoreGrid + BLOCK) / BLOCK;  // covers entries 0..R inclusive
    uint32_t va[PER_T], vc[PER_T];
    uint32_t ma = 0, mc = 0;
#pragma unroll
    for (int k = 0; k < PER_T; ++k) {
        const int i = tid * PER_T + k;
        va[k] = i < R ? ld(p.seg_arcs + i) : 0u;
        vc[k] = i < R ? ld(p.seg_cnt + i) : 0u;
        ma += va[k];
        mc += vc[k];
    }
    uint32_t ea, ec;
    block_excl_scan<BLOCK>(ma, ea, sh.tmp);
    block_excl_scan<BLOCK>(mc, ec, sh.tmp);
#pragma unroll
    for (int k = 0; k < PER_T; ++k) {
        const int i = tid * PER_T + k;
        if (i <= R) {
            sh.x.big.segpre[i] = ea;
            sh.x.big.cntpre[i] = ec;
        }
        ea += va[k];
        ec += vc[k];
    }
    __syncthreads();
    return sh.x.big.cntpre[R];
}

// Dense index of the listed row holding arc a (level-wide numbering, a below
// the level's total): its segment by the arc prefix, then its index inside the
// segment by the stored arc offsets. One thread.
template <int BLOCK>
__device__ __forceinline__ uint32_t big_row_at(const SingleParams& p, const ExpandShared<BLOCK>& sh, int64_t a) {
    // Last segment starting at or before a; as a < total, the next segment
    // starts after a, so this one holds arcs.
    int lo = 0, hi = p.restore_grid - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)sh.x.big.segpre[mid] <= a)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int64_t local = a - (int64_t)sh.x.big.segpre[lo];
    const int first = p.seg_start[lo];
    int l2 = 0, h2 = (int)(sh.x.big.cntpre[lo + 1] - sh.x.big.cntpre[lo]) - 1;
    while (l2 < h2) {
        const int mid = (l2 + h2 + 1) >> 1;
        if ((int64_t)ld(p.bl_pre + first + mid) <= local)
            l2 = mid;
        else
            h2 = mid - 1;
    }
    return sh.x.big.cntpre[lo] + (uint32_t)l2;
}

// Listed row d (dense numbering across segments): its vertex and its first arc
// in the level-wide numbering.
template <int BLOCK>
__device__ __forceinline__ void big_row(const SingleParams& p, const ExpandShared<BLOCK>& sh, uint32_t d, int32_t& u,
                                        int64_t& start) {
    int lo = 0, hi = p.restore_grid - 1;  // last segment whose first row is <= d (non-empty by construction)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sh.x.big.cntpre[mid] <= d)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int slot = p.seg_start[lo] + (int)(d - sh.x.big.cntpre[lo]);
    u = ld(p.bl_u + slot);
    start = (int64_t)sh.x.big.segpre[lo] + ld(p.bl_pre + slot);
}

// The general claim on already-gathered heads v (lanes with ok set): global
// filter, confirmation on the level array, claim.
template <bool kAtomic, int U>
__device__ __forceinline__ void visit_out(const SingleParams& p, const int32_t (&v)[U], const bool (&ok)[U],
                                          const int32_t (&par)[U], int lvl) {
#pragma unroll
    for (int i = 0; i < U; ++i) {
        const uint32_t b = 1u << (v[i] & 31);
        if (!ok[i]) continue;
        if (kAtomic) {
            if (!(atomicOr(p.vis + (v[i] >> 5), b) & b)) record(p, v[i], lvl, par[i]);
        } else {
            const uint32_t w = p.vis[v[i] >> 5];
            if (!(w & b) && ld(p.lv + lv_at(p, v[i])) == -1) {
                p.vis[v[i] >> 5] = w | b;  // may lose a concurrent update: restored later
                record(p, v[i], lvl, par[i]);
            }
        }
    }
}

// Visit of arcs whose heads all lie in the destination block held in LDS
// (words [w0, w0 + nw) of the visited bitmap, exact at the start of the
// level): a set bit is final; a clear one is claimed in LDS first (one claim
// per workgroup and vertex), then on the global visited word. With
// update_mode 1 that global claim is an atomicOr at workgroup scope: it
// executes in the L2 of this XCD, where every workgroup of this block runs
// (workgroups go to the eight XCDs in turn and pairs are numbered to match),
// so it is exact among them, cheap, and a lost race with another XCD (there
// is none for in-block arcs when the assignment holds) only makes a
// duplicate claim of the same level, which the restoration pass tolerates.
// With update_mode 2 it is a device-scope atomicOr. A claim needs no
// confirmation on the level array: the LDS bits already exclude every vertex
// of an earlier level. An arc outside the block (none, when the grouping
// holds) takes the confirmed path of visit_arcs.
template <bool kAtomic, int U>
__device__ __forceinline__ void visit_blocked(const SingleParams& p, const int64_t (&pos)[U], const bool (&ok)[U],
                                              const int32_t (&par)[U], int lvl, uint32_t* bits, uint32_t w0,
                                              uint32_t nw) {
    int32_t v[U];
#pragma unroll
    for (int i = 0; i < U; ++i) v[i] = __builtin_nontemporal_load(p.col + pos[i]);
    uint32_t lw[U];
    bool in[U];
#pragma unroll
    for (int i = 0; i < U; ++i) {
        const uint32_t wi = ((uint32_t)v[i] >> 5) - w0;
        in[i] = wi < nw;
        lw[i] = bits[in[i] ? wi : 0u];
    }
    bool cand[U], any_out = false;
#pragma unroll
    for (int i = 0; i < U; ++i) {
        const uint32_t b = 1u << (v[i] & 31);
        cand[i] = ok[i] & !(in[i] & ((lw[i] & b) != 0u));
        if (cand[i] & in[i]) cand[i] = (atomicOr(bits + (((uint32_t)v[i] >> 5) - w0), b) & b) == 0u;
        any_out |= cand[i] & !in[i];
    }
#pragma unroll
    for (int i = 0; i < U; ++i) {
        const uint32_t b = 1u << (v[i] & 31);
        if (cand[i] & in[i]) {
            const uint32_t old = kAtomic ? atomicOr(p.vis + (v[i] >> 5), b)
                                         : __hip_atomic_fetch_or(p.vis + (v[i] >> 5), b, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
            if (!(old & b)) record(p, v[i], lvl, par[i]);
        }
    }
    if (__ballot(any_out)) {
        // Heads outside the block: the general visit (global filter, level
        // confirmation, claim), for the lanes that hold such an arc.
        bool out[U];
#pragma unroll
        for (int i = 0; i < U; ++i) out[i] = cand[i] & !in[i];
        visit_out<kAtomic, U>(p, v, out, par, lvl);
    }
}

// Visit of arcs at a hub level: each head goes, with its parent, to the bin
// of its restore chunk, in this workgroup's region of that bin (position from
// the workgroup's LDS counter); the restoration pass claims them. A region
// that is full sends further heads down the general claim path.
template <bool kAtomic, int U>
__device__ __forceinline__ void visit_binned(const SingleParams& p, const int64_t (&pos)[U], const bool (&ok)[U],
                                             const int32_t (&par)[U], int lvl, uint32_t* cnt, uint32_t wg) {
    int32_t v[U];
#pragma unroll
    for (int i = 0; i < U; ++i) v[i] = __builtin_nontemporal_load(p.col + pos[i]);
    bool over[U], any_over = false;
#pragma unroll
    for (int i = 0; i < U; ++i) {
        over[i] = false;
        if (ok[i]) {
            const uint32_t b = (uint32_t)v[i] >> kBinShift;
            const uint32_t q = atomicAdd(cnt + b, 1u);
            if (q < (uint32_t)p.bin_k) {
                p.bin_e[((int64_t)b * p.bin_groups + wg) * p.bin_k + q] = make_int2(v[i], par[i]);
            } else {
                over[i] = true;
                any_over = true;
            }
        }
    }
    if (__ballot(any_over)) visit_out<kAtomic, U>(p, v, over, par, lvl);
}

// Wavefront walk over staged rows: arcs [from, hi_arc) of a numbering in which
// staged row r starts at sh.x.big.start[r] (non-decreasing; empty rows share
// their successor's start) and its arc a sits at column index base[r] + a.
// Each wavefront takes a contiguous run, 64 x kBigUnroll consecutive arcs per
// step, so column reads are coalesced. The row boundaries inside a step come
// from one LDS read per lane (the next 64 staged starts) and a ballot; rows
// are long, so a step crosses at most a few, and no lane runs a search or a
// loop of its own.
template <bool kAtomic, int BLOCK, int kMode>
__device__ __forceinline__ void walk_staged(const SingleParams& p, ExpandShared<BLOCK>& sh, int64_t from,
                                            int64_t hi_arc, int nt, int lvl, const LdsVis& lds, uint32_t* bits,
                                            uint32_t w0, uint32_t nw) {
    constexpr int NW = BLOCK / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t per_w = ((hi_arc - from + NW - 1) / NW + 63) & ~(int64_t)63;
    const int64_t w_lo = from + (int64_t)wid * per_w;
    const int64_t w_hi = w_lo + per_w < hi_arc ? w_lo + per_w : hi_arc;
    if (w_lo >= w_hi) return;
    int lo = 0, hi = nt - 1;  // last staged row starting at or before w_lo
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sh.x.big.start[mid] <= w_lo) lo = mid; else hi = mid - 1;
    }
    int row = lo;  // the same in every lane
    constexpr int SPAN = 64 * kBigUnroll;
    for (int64_t ws = w_lo; ws < w_hi; ws += SPAN) {
        // The next 64 staged row starts, one per lane: those inside this span
        // are the row boundaries the span crosses (sorted).
        const int nr = row + 1 + lane;
        const int64_t x = nr < nt ? sh.x.big.start[nr] : INT64_MAX;
        const uint64_t inside = __ballot(x < ws + SPAN);
        const int k = __popcll(inside);  // boundaries before the span's end, all in lanes 0..k-1
        int64_t pos[kBigUnroll];
        bool ok[kBigUnroll];
        int32_t par[kBigUnroll];
        int r[kBigUnroll];
#pragma unroll
        for (int i = 0; i < kBigUnroll; ++i) r[i] = row;
        int next_row;
        if (k < 64) {
            for (int j = 0; j < k; ++j) {  // the same trip count in every lane
                const int64_t bj = shfl64(x, j);
#pragma unroll
                for (int i = 0; i < kBigUnroll; ++i) {
                    const int64_t a = ws + i * 64 + lane;
                    r[i] += (a < w_hi ? a : w_hi - 1) >= bj ? 1 : 0;
                }
            }
            next_row = row + __popcll(__ballot(x <= ws + SPAN));
        } else {
            // More than 64 rows in one span: each lane moves its own cursor.
#pragma unroll
            for (int i = 0; i < kBigUnroll; ++i) {
                const int64_t a = ws + i * 64 + lane;
                const int64_t ac = a < w_hi ? a : w_hi - 1;
                int rr = i == 0 ? row : r[i - 1];
                while (rr + 1 < nt && sh.x.big.start[rr + 1] <= ac) ++rr;
                r[i] = rr;
            }
            next_row = __shfl(r[kBigUnroll - 1], 63, 64);
            while (next_row + 1 < nt && sh.x.big.start[next_row + 1] <= ws + SPAN) ++next_row;
        }
#pragma unroll
        for (int i = 0; i < kBigUnroll; ++i) {
            const int64_t a = ws + i * 64 + lane;
            ok[i] = a < w_hi;
            const int64_t ac = ok[i] ? a : w_hi - 1;
            pos[i] = sh.x.big.base[r[i]] + ac;
            par[i] = sh.x.big.u[r[i]];
        }
        row = next_row;  // the row of the next span's first arc
        if (kMode == kWalkBlocked)
            visit_blocked<kAtomic, kBigUnroll>(p, pos, ok, par, lvl, bits, w0, nw);
        else if (kMode == kWalkBinned)
            visit_binned<kAtomic, kBigUnroll>(p, pos, ok, par, lvl, bits, w0);
        else
            visit_arcs<kAtomic, kBigUnroll>(p, pos, ok, par, lvl, lds);
    }
}

// Rows above T2: this workgroup's share [a0, a1) of the level's concatenated
// big-row arcs. Row metadata is staged BLOCK rows at a time (every thread
// loads one row); the wavefronts then walk the staged arcs.
template <typename OffT, bool kAtomic, int BLOCK, int kMode = kWalkProbe>
__device__ __forceinline__ void expand_big(const SingleParams& p, ExpandShared<BLOCK>& sh, int64_t a0, int64_t a1,
                                           int lvl, unsigned long long& arcs, const LdsVis& lds,
                                           uint32_t* bin_counts = nullptr) {
    const int tid = threadIdx.x;
    const uint32_t total_rows = big_prefix<BLOCK>(p, sh);
    if (tid == 0) sh.row0 = big_row_at<BLOCK>(p, sh, a0);
    __syncthreads();
    uint32_t d0 = sh.row0;
    int64_t from = a0;
    while (from < a1 && d0 < total_rows) {
        // Stage rows d0 .. d0+BLOCK-1.
        const uint32_t d = d0 + (uint32_t)tid;
        const int nt = (int)min((uint32_t)BLOCK, total_rows - d0);
        int64_t end = a1;
        if (tid < nt) {
            int32_t u;
            int64_t start;
            big_row<BLOCK>(p, sh, d, u, start);
            const int64_t beg = load_off<OffT>(p.off, u);
            const int64_t deg = load_off<OffT>(p.off, (int64_t)u + 1) - beg;
            sh.x.big.start[tid] = start > from ? start : from;
            sh.x.big.base[tid] = beg - start;
            sh.x.big.u[tid] = out_id(p, u);
            end = start + deg < a1 ? start + deg : a1;
        }
        if (tid == nt - 1) sh.staged_end = end;
        __syncthreads();
        const int64_t hi_arc = sh.staged_end;
        walk_staged<kAtomic, BLOCK, kMode>(p, sh, from, hi_arc, nt, lvl, lds, bin_counts, (uint32_t)blockIdx.x, 0u);
        if (tid == 0) arcs += (unsigned long long)(hi_arc - from);
        from = hi_arc;
        d0 += (uint32_t)nt;
        __syncthreads();
    }
}

// Rows above T2 at a hub level, into the destination bins: every workgroup
// (with a share or not) zeroes its LDS counters (one per bin), walks its share,
// and writes how many entries each of its regions received, so the
// restoration pass can read every region of a bin.
template <typename OffT, bool kAtomic, int BLOCK>
__device__ __forceinline__ void expand_big_binned(const SingleParams& p, ExpandShared<BLOCK>& sh, int64_t a0,
                                                  int64_t a1, int lvl, unsigned long long& arcs, uint32_t* counts) {
    const int tid = threadIdx.x;
    for (int b = tid; b < p.bin_nb; b += BLOCK) counts[b] = 0u;
    __syncthreads();
    if (a0 < a1) expand_big<OffT, kAtomic, BLOCK, kWalkBinned>(p, sh, a0, a1, lvl, arcs, LdsVis::none(counts), counts);
    __syncthreads();
    uint32_t* mine = p.bin_cnt + (int64_t)blockIdx.x * p.bin_nb;
    for (int b = tid; b < p.bin_nb; b += BLOCK) mine[b] = min(counts[b], (uint32_t)p.bin_k);
}

// Rows above T2 on the degree-ordered copy, whose arcs are grouped by
// destination block: the level's big-row arcs are cut into C chunks, and the
// pair (block b, chunk c) goes to one workgroup, which loads block b's visited
// bits (exact at level start) into LDS and walks, in every staged row of chunk
// c, only the arcs that fall in block b (a contiguous run of the row, from the
// row's block offsets). Every probe of such an arc is answered in LDS. Pairs
// are numbered so that the workgroups of one block run on one XCD (workgroups
// go to the eight XCDs in turn), where they share the L2 lines of the
// block's global visited words.
template <typename OffT, bool kAtomic, int BLOCK>
__device__ __forceinline__ void expand_blocked(const SingleParams& p, ExpandShared<BLOCK>& sh, int64_t ta, int lvl,
                                               unsigned long long& arcs, uint32_t* bits) {
    const int tid = threadIdx.x;
    const int64_t G = gridDim.x;
    const int B = p.nblk;
    const int64_t C = G >= B ? G / B : 1;
    const int64_t SW = (int64_t)1 << (p.blk_shift - 5);  // visited words per block (a multiple of 64)
    const uint32_t total_rows = big_prefix<BLOCK>(p, sh);
    for (int64_t pair = blockIdx.x; pair < (int64_t)B * C; pair += G) {
        const int b = (int)(pair % B);
        const int64_t c = pair / B;
        const int64_t a0 = ta * c / C, a1 = ta * (c + 1) / C;
        if (a0 >= a1) continue;
        const int64_t w0 = (int64_t)b * SW;
        const int64_t nw = SW < p.words - w0 ? SW : p.words - w0;  // multiple of 64
        __syncthreads();  // the previous pair's probes are done with the LDS bits
        {
            const unsigned long long* src = reinterpret_cast<const unsigned long long*>(p.vis_prev + w0);
            unsigned long long* dst = reinterpret_cast<unsigned long long*>(bits);
            for (int64_t i = tid; i < nw / 2; i += BLOCK) dst[i] = ld(src + i);
        }
        if (tid == 0) sh.row0 = big_row_at<BLOCK>(p, sh, a0);
        __syncthreads();
        uint32_t d0 = sh.row0;
        int64_t from = a0;
        while (from < a1 && d0 < total_rows) {
            // Stage rows d0 .. d0+BLOCK-1: the part of each row inside the
            // chunk and block b, renumbered consecutively.
            const uint32_t d = d0 + (uint32_t)tid;
            const int nt = (int)min((uint32_t)BLOCK, total_rows - d0);
            int64_t end = a1;
            uint32_t len = 0;
            int64_t col0 = 0;
            int32_t uo = 0;
            if (tid < nt) {
                int32_t u;
                int64_t start;
                big_row<BLOCK>(p, sh, d, u, start);
                const int64_t beg = load_off<OffT>(p.off, u);
                const int64_t deg = load_off<OffT>(p.off, (int64_t)u + 1) - beg;
                const int64_t lo = (from > start ? from : start) - start;
                const int64_t hi = (a1 < start + deg ? a1 : start + deg) - start;
                uint32_t rk = 0;
                const bool listed = hot_slot((uint32_t)u, (uint32_t)p.hot_span, (uint32_t)p.hot_shift, rk) &&
                                    rk < (uint32_t)p.bseg_rows;
                // A row without block offsets (none, when the tables agree)
                // is walked whole by the pairs of block 0, on the confirmed path.
                int64_t sb = 0, se = b == 0 ? deg : 0;
                if (listed) {
                    const uint32_t* sg = p.bseg + (size_t)rk * (size_t)(B + 1);
                    sb = sg[b];
                    se = sg[b + 1];
                }
                const int64_t elo = lo > sb ? lo : sb, ehi = hi < se ? hi : se;
                if (ehi > elo) {
                    len = (uint32_t)(ehi - elo);
                    col0 = beg + elo;
                }
                uo = out_id(p, u);
                end = start + deg < a1 ? start + deg : a1;
            }
            if (tid == nt - 1) sh.staged_end = end;
            uint32_t excl;
            const uint32_t tot = block_excl_scan<BLOCK>(len, excl, sh.tmp);
            if (tid < nt) {
                sh.x.big.start[tid] = excl;
                sh.x.big.base[tid] = col0 - (int64_t)excl;
                sh.x.big.u[tid] = uo;
            }
            __syncthreads();
            walk_staged<kAtomic, BLOCK, kWalkBlocked>(p, sh, 0, tot, nt, lvl, LdsVis::none(bits), bits,
                                                      (uint32_t)w0, (uint32_t)nw);
            if (tid == 0) arcs += (unsigned long long)tot;
            from = sh.staged_end;
            d0 += (uint32_t)nt;
            __syncthreads();
        }
    }
}

// One bottom-up level (the direction-optimising hybrid): every vertex not yet
// visited scans its neighbours and takes the first one in the frontier as its
// parent, at level lvl. Each wavefront owns a contiguous run of visited words;
// it compacts the unvisited vertices of 64 words at a time into its LDS ring,
// gives one vertex to each lane, and collects the new bits of those 64 words
// in LDS. The lane that owns a word then writes it once (vis = snapshot | new
// bits), which marks it for the restoration pass. The frontier is read with
// device-scope loads: another XCD wrote it in the previous launch.
template <typename OffT, int BLOCK>
__device__ __forceinline__ void bottom_up(const SingleParams& p, ExpandShared<BLOCK>& sh, int lvl,
                                          const LdsVis& lds, bool cold_empty) {
    // Is u in the frontier? From the LDS copy of the frontier's bits (hot ids,
    // or whole words) where it holds u; otherwise from the frontier bitmap,
    // unless the frontier has no vertex outside the hot set.
    auto in_frontier = [&](int32_t u) -> bool {
        uint32_t bit;
        if (lds_slot(lds, u, bit)) return (lds.bits[bit >> 5] >> (bit & 31)) & 1u;
        if (cold_empty) return false;
        return (ld(p.fr + ((uint32_t)u >> 5)) >> (u & 31)) & 1u;
    };
    constexpr int NW = BLOCK / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t waves = (int64_t)gridDim.x * NW;
    const int64_t gw = (int64_t)blockIdx.x * NW + wid;
    const int64_t wpw = (p.words + waves - 1) / waves;
    const int64_t w0 = gw * wpw;
    const int64_t w1 = w0 + wpw < p.words ? w0 + wpw : p.words;
    uint32_t* ring = sh.x.w.ring[wid];
    uint32_t* bits = sh.x.w.bu_bits[wid];
    for (int64_t base = w0; base < w1; base += 64) {
        const int64_t wi = base + lane;
        uint32_t prev = ~0u, nz = 0u;
        if (wi < w1) {
            prev = ld(p.vis_prev + wi);
            nz = p.nzmap[wi];
        }
        uint32_t word = ~prev & nz;  // vertices without arcs cannot be reached: skip them
        const int64_t first_v = wi * 32;
        if (wi >= w1 || first_v >= p.n)
            word = 0;
        else if (first_v + 32 > p.n)
            word &= (1u << (p.n - first_v)) - 1u;  // ids beyond n do not exist
        bits[lane] = 0u;
        uint32_t head = 0, tail = 0;
        while (true) {
            const bool has = word != 0;
            const uint64_t m = __ballot(has);
            const bool flush = m == 0;
            if (has) {
                const int b = __builtin_ctz(word);
                word &= word - 1;
                ring[(tail + rank_in(m)) & 127] = (uint32_t)(wi * 32 + b);
            }
            tail += __popcll(m);
            while (tail - head >= 64 || (flush && tail != head)) {
                const uint32_t cnt = tail - head < 64 ? tail - head : 64;
                const bool valid = (uint32_t)lane < cnt;
                const int32_t v = valid ? (int32_t)ring[(head + lane) & 127] : 0;
                head += cnt;
                // Phase 1: each lane checks the first kBuFirst arcs of its vertex
                // (independent loads); most vertices settle here.
                int32_t par = -1;
                int64_t b = 0, e = 0;
                if (valid) {
                    b = load_off<OffT>(p.off, v);
                    e = load_off<OffT>(p.off, (int64_t)v + 1);
                    int32_t u[kBuFirst];
                    bool f[kBuFirst];
#pragma unroll
                    for (int k = 0; k < kBuFirst; ++k) u[k] = b + k < e ? p.col[b + k] : -1;
#pragma unroll
                    for (int k = 0; k < kBuFirst; ++k) f[k] = u[k] >= 0 && in_frontier(u[k]);
#pragma unroll
                    for (int k = 0; k < kBuFirst; ++k)
                        if (par < 0 && f[k]) par = u[k];
                }
                // Phase 2: longer rows without a hit are scanned by the whole
                // wavefront, 64 arcs at a time, until the first frontier neighbour.
                uint64_t longm = __ballot(valid && par < 0 && e - b > kBuFirst);
                while (longm) {
                    const int src = __builtin_ctzll(longm);
                    longm &= longm - 1;
                    const int64_t lb = shfl64(b, src) + kBuFirst, le = shfl64(e, src);
                    int32_t found = -1;
                    for (int64_t j0 = lb; j0 < le && found < 0; j0 += 64) {
                        const int64_t j = j0 + lane;
                        const int32_t u = j < le ? p.col[j] : -1;
                        const bool hit = u >= 0 && in_frontier(u);
                        const uint64_t hm = __ballot(hit);
                        if (hm) found = __shfl(u, __builtin_ctzll(hm), 64);
                    }
                    if (lane == src) par = found;
                }
                if (par >= 0) {
                    record(p, v, lvl + 1, out_id(p, par));
                    atomicOr(bits + ((v >> 5) - base), 1u << (v & 31));
                }
            }
            if (flush) break;
        }
        const uint32_t nb = bits[lane];
        if (nb) st(p.vis + wi, prev | nb);
    }
}

// a0: levels/parents = -1, bitmaps cleared, root seeded, counters reset.
template <typename OffT, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_init(SingleParams p, int nslots) {
    const int64_t gtid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t gsize = (int64_t)gridDim.x * BLOCK;
    const int ro = p.root_out;
    if (p.new2old) {
        // Degree-ordered copy: the run's {level, parent} records (the caller's
        // arrays are written after the last level). Two records per 16 bytes.
        int4* r4 = reinterpret_cast<int4*>(p.lv);
        const int64_t n2 = p.n / 2;
        for (int64_t i = gtid; i < n2; i += gsize) {
            int4 x = make_int4(-1, -1, -1, -1);
            if ((p.root >> 1) == i) {
                if (p.root & 1) { x.z = 0; x.w = ro; } else { x.x = 0; x.y = ro; }
            }
            r4[i] = x;
        }
        if ((p.n & 1) && gtid == 0) {
            const int64_t v = p.n - 1;
            p.lv[2 * v] = (v == p.root) ? 0 : -1;
            p.lv[2 * v + 1] = (v == p.root) ? ro : -1;
        }
    } else {
        // The caller's levels and parents (caller ids).
        const int64_t n4 = p.n / 4;
        const bool aligned = ((reinterpret_cast<uintptr_t>(p.out_lv) | reinterpret_cast<uintptr_t>(p.out_pa)) & 15) == 0;
        if (aligned) {
            int4* lv4 = reinterpret_cast<int4*>(p.out_lv);
            int4* pa4 = reinterpret_cast<int4*>(p.out_pa);
            for (int64_t i = gtid; i < n4; i += gsize) {
                int4 a = make_int4(-1, -1, -1, -1), b = make_int4(-1, -1, -1, -1);
                if ((ro >> 2) == i) {
                    const int k = ro & 3;
                    if (k == 0) { a.x = 0; b.x = ro; }
                    if (k == 1) { a.y = 0; b.y = ro; }
                    if (k == 2) { a.z = 0; b.z = ro; }
                    if (k == 3) { a.w = 0; b.w = ro; }
                }
                lv4[i] = a;
                pa4[i] = b;
            }
        }
        for (int64_t i = (aligned ? n4 * 4 : 0) + gtid; i < p.n; i += gsize) {
            p.out_lv[i] = (i == ro) ? 0 : -1;
            p.out_pa[i] = (i == ro) ? ro : -1;
        }
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
    uint32_t rs = 0;
    const bool root_hot = p.hot_words > 0 && hot_slot((uint32_t)p.root, (uint32_t)p.hot_span, (uint32_t)p.hot_shift, rs);
    for (int64_t i = gtid; i < p.hot_words; i += gsize) {
        const uint32_t x = (root_hot && i == (rs >> 5)) ? 1u << (rs & 31) : 0u;
        p.hot_vis[i] = x;
        p.hot_fr[i] = x;
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
        // The first frontier: the root, listed below with the arcs of its row.
        unsigned long long* sp = stripe(p.ctrl, (int)(i / kStripes), (int)(i % kStripes));
        sp[0] = (i == 0) ? 1ull : 0ull;
        sp[1] = (i == 0) ? (unsigned long long)root_deg : 0ull;
        sp[2] = (i == 0) ? 1ull : 0ull;
        p.ctrl->bigarcs[i / kStripes][(i % kStripes) * kStripeStride] = (i == 0 && root_big) ? (unsigned long long)root_deg : 0ull;
    }
    if (gtid == 0) {
        p.ctrl->done = 0;
        p.ctrl->num_levels = 0;
        p.ctrl->reached = 0;
        p.ctrl->arcs = 0;
        p.ctrl->dir[0] = 0;
        p.ctrl->dir[1] = 0;
        p.ctrl->visited[0] = 0;
        p.ctrl->visited[1] = 0;
        p.ctrl->steps = 0;
        p.ctrl->shift[0] = 0;
        p.ctrl->shift[1] = 0;
    }
    // The first frontier, listed for the small-level path: the root alone.
    for (int64_t i = gtid; i < p.restore_grid; i += gsize) {
        p.sl_cnt[i] = i == 0 ? 1 : 0;
        if (i == 0) p.sl[0] = p.root;
    }
}

// After the last level on the degree-ordered copy: the caller's levels and
// parents from the run's records, in caller order. The writes are coalesced;
// cold ids keep the caller's order, so the record reads are nearly coalesced
// too, and only the hot vertices' records are gathered one by one (a random
// read costs one line, a random partial-line write a fetch and a write-back).
__global__ __launch_bounds__(256) void k_out(const unsigned long long* rec, const int32_t* old2new, int32_t* out_lv,
                                             int32_t* out_pa, int64_t n) {
    const int64_t gsize = (int64_t)gridDim.x * 256;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += gsize) {
        const unsigned long long r = ld(rec + old2new[c]);  // {level, parent}, written by earlier launches
        out_lv[c] = (int32_t)(uint32_t)r;
        out_pa[c] = (int32_t)(uint32_t)(r >> 32);
    }
}

// Row starts (beg) and exclusive arc prefix (pre) of a small-level list of nf
// ids (nf <= kSmallMax); returns the list's arcs. A thread owns PER
// consecutive entries. Its sum is clamped above s_arcs, so the total stays in
// 32 bits and exceeds s_arcs exactly when the true total does (the prefix is
// then not used).
template <typename OffT, int BLOCK>
__device__ __forceinline__ uint32_t small_prefix(const SingleParams& p, ExpandShared<BLOCK>& sh, const int32_t* list,
                                                 uint32_t nf, int64_t* beg, uint32_t* pre) {
    constexpr int PER = kSmallMax / BLOCK;
    const int tid = threadIdx.x;
    int64_t d[PER];
    uint64_t mine = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = tid * PER + k;
        d[k] = 0;
        if (i < (int)nf) {
            const int32_t u = list[i];
            const int64_t b = load_off<OffT>(p.off, u);
            beg[i] = b;
            d[k] = load_off<OffT>(p.off, (int64_t)u + 1) - b;
        }
        mine += (uint64_t)d[k];
    }
    const uint32_t cap = (uint32_t)p.s_arcs + 1u;
    uint32_t at;
    const uint32_t total = block_excl_scan<BLOCK>(mine < cap ? (uint32_t)mine : cap, at, sh.tmp);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = tid * PER + k;
        if (i < (int)nf) pre[i] = at;
        at += (uint32_t)d[k];
    }
    __syncthreads();
    return total;
}

// Small levels (tunable sparse_frontier, s_max > 0), run by workgroup 0 of an
// expansion whose frontier the previous restore listed in full (at most s_max
// vertices with at most s_arcs arcs; a restore block with at most kSmallSeg
// new vertices lists them and counts them and their rows' arcs). Arcs are spread over the
// threads, claims are exact (atomicOr on the visited word: no other
// workgroup runs), and the next frontier is listed in LDS. While it stays
// small the loop goes on to the next level itself, after taking the frontier
// into the snapshot (and the hot bits). It stops at:
//  * an empty next frontier: the run is done;
//  * a large next frontier: the level it just expanded is left to this
//    step's restore, exactly as the grid expansion leaves a level (claims
//    recorded, visited bits set, the snapshot unchanged), and the levels it
//    ran beyond its own go into the next step's shift.
// LDS (the expansion's dynamic region): two lists, the row starts and the
// arc prefix of kSmallMax entries each (20 bytes an entry).
template <typename OffT, int BLOCK>
__device__ void small_levels(const SingleParams& p, ExpandShared<BLOCK>& sh, uint32_t* dyn, int lvl, int step) {
    constexpr int PR = (kMaxRestoreGrid + BLOCK - 1) / BLOCK;  // restore blocks per thread
    int32_t* list[2] = {reinterpret_cast<int32_t*>(dyn), reinterpret_cast<int32_t*>(dyn) + kSmallMax};
    int64_t* beg = reinterpret_cast<int64_t*>(dyn + 2 * kSmallMax);
    uint32_t* pre = dyn + 4 * kSmallMax;
    const int tid = threadIdx.x;
    const int shift0 = sh.shift;
    unsigned long long seen = sh.seen;

    // The frontier from the restore blocks' lists, in block order.
    const int R = p.restore_grid;
    int cb[PR];
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < PR; ++k) {
        const int r = tid * PR + k;
        const int c = r < R ? ld(p.sl_cnt + r) : 0;
        cb[k] = c < kSmallSeg ? c : kSmallSeg;  // all of them: every block listed all it found
        mine += (uint32_t)cb[k];
    }
    uint32_t ex;
    uint32_t nf = block_excl_scan<BLOCK>(mine, ex, sh.tmp);
#pragma unroll
    for (int k = 0; k < PR; ++k) {
        const int r = tid * PR + k;
        for (int j = 0; j < cb[k]; ++j)
            if (ex + j < (uint32_t)kSmallMax) list[0][ex + j] = ld(p.sl + (int64_t)r * kSmallSeg + j);
        ex += (uint32_t)cb[k];
    }
    if (nf > (uint32_t)kSmallMax) nf = kSmallMax;  // not reached: nf equals the frontier count, at most s_max
    __syncthreads();

    unsigned long long arcs_done = 0, reached_done = 0;  // this launch's statistics (thread 0)
    int cur = 0, k_beyond = 0;
    // Row starts and the exclusive arc prefix of the current list; the arcs
    // the loop checks are at most s_arcs (the counts checked before the first
    // level, this pass before the others).
    uint32_t arcs = small_prefix<OffT, BLOCK>(p, sh, list[0], nf, beg, pre);
    while (true) {
        if (tid == 0) sh.s_next = 0;
        __syncthreads();
        // Expand: arc a belongs to the last entry whose prefix is at most a.
        // The claim is the atomicOr itself (no other workgroup runs).
        int32_t* nxt = list[cur ^ 1];
        for (uint32_t a = tid; a < arcs; a += BLOCK) {
            int lo = 0, hi = (int)nf - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (pre[mid] <= a) lo = mid; else hi = mid - 1;
            }
            const int32_t u = list[cur][lo];
            const int32_t v = p.col[beg[lo] + (a - pre[lo])];
            const uint32_t bit = 1u << (v & 31);
            if (!(atomicOr(p.vis + ((uint32_t)v >> 5), bit) & bit)) {
                record(p, v, lvl + 1, out_id(p, u));
                const uint32_t k = atomicAdd(&sh.s_next, 1u);
                if (k < (uint32_t)kSmallMax) nxt[k] = v;
            }
        }
        __syncthreads();
        const uint32_t nn = sh.s_next;
        if (tid == 0) arcs_done += arcs;
        if (p.hybrid && tid == 0) {
            st(&p.ctrl->dir[(lvl + 1) & 1], 0);
            st(&p.ctrl->visited[(lvl + 1) & 1], seen + nf);
        }
        seen += nf;
        if (nn == 0) {  // nothing new: level lvl + 1 is empty and the run is done
            if (tid == 0) {
                st(p.arcs_slot, ld(p.arcs_slot) + arcs_done);
                st(p.reached_slot, ld(p.reached_slot) + reached_done);
                p.ctrl->num_levels = lvl + 1;
                p.ctrl->steps = step + 1;
                __hip_atomic_store(&p.ctrl->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            return;
        }
        // Is the next frontier small too (vertices, then arcs)? Its row starts
        // and arc prefix replace the current ones (the expansion is over).
        bool go_on = nn <= (uint32_t)p.s_max;
        if (go_on) {
            arcs = small_prefix<OffT, BLOCK>(p, sh, nxt, nn, beg, pre);
            go_on = arcs <= (uint32_t)p.s_arcs;
        }
        if (!go_on) {
            // Leave level lvl to this step's restore: the next level's counters
            // start at zero as an expansion would have set them.
            if (tid < kStripes) {
                unsigned long long* sp = stripe(p.ctrl, (lvl + 1) & 1, tid);
                st(sp, 0ull);
                st(sp + 1, 0ull);
                st(sp + 2, 0ull);
                st(&p.ctrl->bigarcs[(lvl + 1) & 1][tid * kStripeStride], 0ull);
            }
            if (tid == 0) {
                st(p.arcs_slot, ld(p.arcs_slot) + arcs_done);
                st(p.reached_slot, ld(p.reached_slot) + reached_done);
                st(&p.ctrl->shift[(step + 1) & 1], shift0 + k_beyond);
            }
            return;
        }
        // The next frontier stays here: the snapshot and the hot bits take it in.
        for (uint32_t i = tid; i < nn; i += BLOCK) {
            const int32_t v = nxt[i];
            atomicOr(p.vis_prev + ((uint32_t)v >> 5), 1u << (v & 31));
            uint32_t r;
            if (p.hot_words > 0 && hot_slot((uint32_t)v, (uint32_t)p.hot_span, (uint32_t)p.hot_shift, r))
                atomicOr(p.hot_vis + (r >> 5), 1u << (r & 31));
        }
        if (tid == 0) reached_done += nn;
        cur ^= 1;
        nf = nn;
        ++lvl;
        ++k_beyond;
    }
}

// Expansion of level `lvl` (frontier bitmap p.fr).
template <typename OffT, int BLOCK, bool kAtomic>
__global__ __launch_bounds__(BLOCK) void k_expand(SingleParams p, int lvl_arg) {
    constexpr int NW = BLOCK / 64;
    __shared__ ExpandShared<BLOCK> sh;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t G = gridDim.x, bid = blockIdx.x;
    // Step lvl_arg expands level lvl_arg + shift (small levels on; else shift
    // is 0). Whether the run has ended, the frontier size and the arcs of the
    // frontier's rows above T2 (both counted by the previous restore), the
    // small-level counts and the direction state are all read in one round
    // (small levels are bound by such round trips): both parities, since the
    // level's parity is known only with the shift.
    if (tid < 64) {
        int dn = 0, a = 0, wb[2] = {0, 0};
        unsigned long long sn[2] = {0, 0};
        if (tid == 0) {
            dn = ld(&p.ctrl->done);
            if (p.s_max > 0) a = ld(&p.ctrl->shift[lvl_arg & 1]);
            if (p.hybrid) {
                wb[0] = ld(&p.ctrl->dir[0]);
                wb[1] = ld(&p.ctrl->dir[1]);
                sn[0] = ld(&p.ctrl->visited[0]);
                sn[1] = ld(&p.ctrl->visited[1]);
            }
        }
        const unsigned long long c0 = ld(stripe(p.ctrl, 0, tid)), c1 = ld(stripe(p.ctrl, 1, tid));
        const unsigned long long b0 = ld(&p.ctrl->bigarcs[0][tid * kStripeStride]);
        const unsigned long long b1 = ld(&p.ctrl->bigarcs[1][tid * kStripeStride]);
        unsigned long long sa0 = 0, sa1 = 0, sl0 = 0, sl1 = 0;  // listed arcs and ids
        if (p.s_max > 0) {
            sa0 = ld(stripe(p.ctrl, 0, tid) + 1);
            sa1 = ld(stripe(p.ctrl, 1, tid) + 1);
            sl0 = ld(stripe(p.ctrl, 0, tid) + 2);
            sl1 = ld(stripe(p.ctrl, 1, tid) + 2);
        }
        a = __shfl(a, 0, 64);
        dn = __shfl(dn, 0, 64);
        const int lv = lvl_arg + a, q = lv & 1;
        const unsigned long long c = wave_sum(q ? c1 : c0);
        const unsigned long long b = wave_sum(q ? b1 : b0);
        const unsigned long long sa = p.s_max > 0 ? wave_sum(q ? sa1 : sa0) : 0ull;
        const unsigned long long sl = p.s_max > 0 ? wave_sum(q ? sl1 : sl0) : 0ull;
        if (tid == 0) {
            sh.done = dn;
            sh.lvl = lv;
            sh.shift = a;
            sh.found = c;
            sh.big_total = b;
            sh.was_bu = wb[q];
            sh.seen = sn[q];
            // Small: every new vertex listed, few enough, with few enough arcs.
            sh.small = p.s_max > 0 && sl == c && c <= (unsigned long long)p.s_max &&
                       sa <= (unsigned long long)p.s_arcs;
        }
        if (bid == 0 && !dn) {  // counters for the next level, and the next step's shift
            unsigned long long* sp = stripe(p.ctrl, (lv + 1) & 1, tid);
            st(sp, 0ull);
            st(&p.ctrl->bigarcs[(lv + 1) & 1][tid * kStripeStride], 0ull);
            if (p.s_max > 0) {
                st(sp + 1, 0ull);
                st(sp + 2, 0ull);
                if (tid == 0) st(&p.ctrl->shift[(lvl_arg + 1) & 1], a);
            }
        }
    }
    __syncthreads();
    if (sh.done) return;
    const int lvl = sh.lvl;
    if (sh.found == 0) {
        if (bid == 0 && tid == 0) {
            p.ctrl->num_levels = lvl;
            p.ctrl->steps = lvl_arg + 1;
            __hip_atomic_store(&p.ctrl->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    // ---- a small frontier (a short list with few arcs): workgroup 0 expands
    // it, and the small levels after it, alone; the others leave at once. This
    // comes before the direction choice: the loop rewrites counters that a
    // workgroup starting late reads, and with them it can only see a smaller
    // frontier (or none), which brings it here (or to the return above) too.
    if (sh.small) {
        if (bid == 0) {
            extern __shared__ uint32_t small_lds[];
            small_levels<OffT, BLOCK>(p, sh, small_lds, lvl, lvl_arg);
        }
        return;
    }
    unsigned long long arcs = 0;
    const int64_t ta = (int64_t)sh.big_total;
    // No bins for this level unless its top-down path below decides otherwise.
    if (p.bin_k > 0 && bid == 0 && tid == 0) st(&p.ctrl->binned[lvl & 1], 0);

    // ---- direction (hybrid runs): every workgroup decides the same from the
    // same counters. Bottom-up once the frontier's arcs exceed 1/14 of the arcs
    // still unvisited; back to top-down when the frontier falls below n/24.
    if (p.hybrid) {
        const bool was_bu = sh.was_bu != 0;
        const unsigned long long seen = sh.seen;
        const double nf = (double)sh.found;
        const double mf = (double)ta + nf * ((double)p.nnz / (double)p.n);
        const double unvisited = (double)p.n - (double)seen - nf;
        const double mu = (double)p.nnz * (unvisited > 0.0 ? unvisited : 0.0) / (double)p.n;
        const bool bu = was_bu ? nf * 24.0 >= (double)p.n : mf * 14.0 > mu;
        if (bid == 0 && tid == 0) {
            st(&p.ctrl->dir[(lvl + 1) & 1], bu ? 1 : 0);
            st(&p.ctrl->visited[(lvl + 1) & 1], seen + sh.found);
        }
        if (bu) {
            // LDS copy of the frontier's hot bits, and whether the frontier has
            // any vertex outside the hot set.
            extern __shared__ uint32_t hot_lds[];
            LdsVis lds = LdsVis::none(hot_lds);
            bool cold_empty = false;
            if (p.hot_words > 0) {
                const unsigned long long* src = reinterpret_cast<const unsigned long long*>(p.hot_fr);
                unsigned long long* dst = reinterpret_cast<unsigned long long*>(hot_lds);
                unsigned long long cnt = 0;
                for (int i = tid; i < p.hot_words / 2; i += BLOCK) {
                    const unsigned long long x = ld(src + i);
                    dst[i] = x;
                    cnt += (unsigned long long)__popcll(x);
                }
                cnt = wave_sum(cnt);
                if (lane == 0) sh.red[wid] = cnt;
                __syncthreads();
                unsigned long long hot_in = 0;
                for (int i = 0; i < NW; ++i) hot_in += sh.red[i];
                cold_empty = hot_in == sh.found;
                lds.set_hot((uint32_t)p.hot_span, (uint32_t)p.hot_shift);
                __syncthreads();
            } else if (p.full_words > 0) {
                // The whole frontier bitmap.
                const unsigned long long* src = reinterpret_cast<const unsigned long long*>(p.fr);
                unsigned long long* dst = reinterpret_cast<unsigned long long*>(hot_lds);
                for (int i = tid; i < p.full_words / 2; i += BLOCK) dst[i] = ld(src + i);
                lds.set_words((uint32_t)p.full_words);
                __syncthreads();
            }
            bottom_up<OffT, BLOCK>(p, sh, lvl, lds, cold_empty);
            return;
        }
    }

    extern __shared__ uint32_t hot_lds[];
    const bool large = (int64_t)sh.found >= p.hot_min_frontier;
    // A hub level: few frontier vertices whose rows above T2 carry many arcs,
    // nearly all into unvisited heads. Its big-row heads go to destination bins.
    const bool binned = p.bin_k > 0 && !large && ta >= (int64_t)256 * G;
    if (binned && bid == 0 && tid == 0) st(&p.ctrl->binned[lvl & 1], 1);

    // ---- rows of degree > T2 grouped by destination block (degree-ordered
    // copy, large levels): block by block, the block's visited bits in LDS
    bool big_done = false;
    if (ta > 0 && p.bseg && large && ta >= p.blk_min_arcs) {
        expand_blocked<OffT, kAtomic, BLOCK>(p, sh, ta, lvl + 1, arcs, hot_lds);
        big_done = true;
        __syncthreads();  // the LDS bits are reloaded below
    }

    // ---- LDS copy of visited bits (exact at level start): the compact hot
    // bitmap on the degree-ordered copy, else the whole visited snapshot
    LdsVis lds = LdsVis::none(hot_lds);
    const bool lds_on = large || (!binned && ta >= kHubLdsArcs * G);
    if (p.hot_words > 0 && lds_on) {
        const unsigned long long* src = reinterpret_cast<const unsigned long long*>(p.hot_vis);
        unsigned long long* dst = reinterpret_cast<unsigned long long*>(hot_lds);
        for (int i = tid; i < p.hot_words / 2; i += BLOCK) dst[i] = ld(src + i);
        lds.set_hot((uint32_t)p.hot_span, (uint32_t)p.hot_shift);
        __syncthreads();
    } else if (p.full_words > 0 && lds_on) {
        const unsigned long long* src = reinterpret_cast<const unsigned long long*>(p.vis_prev);
        unsigned long long* dst = reinterpret_cast<unsigned long long*>(hot_lds);
        for (int i = tid; i < p.full_words / 2; i += BLOCK) dst[i] = ld(src + i);
        lds.set_words((uint32_t)p.full_words);
        __syncthreads();
    }

    // ---- rows of degree > T2: the level's big-row arcs, split evenly
    if (ta > 0 && !big_done) {
        int64_t per = (ta + G - 1) / G;
        if (per < p.min_share) per = p.min_share;
        const int64_t a0 = bid * per;
        const int64_t a1 = a0 + per < ta ? a0 + per : ta;
        if (binned) {
            expand_big_binned<OffT, kAtomic, BLOCK>(p, sh, a0, a1, lvl + 1, arcs, hot_lds);
            __syncthreads();  // the word runs below reuse the shared staging
        } else if (a0 < a1) {
            expand_big<OffT, kAtomic, BLOCK>(p, sh, a0, a1, lvl + 1, arcs, lds);
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
                sh.x.w.ring[wid][(tail + rank_in(m)) & 127] = (uint32_t)(wi * 32 + bit);
            }
            tail += __popcll(m);
            if (tail - head >= 64) {
                const int32_t u = (int32_t)sh.x.w.ring[wid][(head + lane) & 127];
                head += 64;
                process_batch<OffT, kAtomic>(p, u, true, lane, lvl + 1, arcs, lds, sh.x.w.starts[wid]);
            }
        }
    }
    if (tail != head) {
        const int cnt = (int)(tail - head);
        const bool valid = lane < cnt;
        const int32_t u = valid ? (int32_t)sh.x.w.ring[wid][(head + lane) & 127] : 0;
        process_batch<OffT, kAtomic>(p, u, valid, lane, lvl + 1, arcs, lds, sh.x.w.starts[wid]);
    }

    // ---- block total of scanned arcs (added to this block's own slot)
    const unsigned long long asum = wave_sum(arcs);
    if (lane == 0) sh.red[wid] = asum;
    __syncthreads();
    if (tid == 0) {
        unsigned long long a = 0;
        for (int i = 0; i < NW; ++i) a += sh.red[i];
        if (a) atomicAdd(p.arcs_slot + bid, a);  // no returned value: nothing to wait for
    }
}

// Restoration of level `lvl`: exact new bits per touched word, visited snapshot,
// next frontier bitmap, the discovered count (striped), and the compacted list
// of the next frontier's rows above T2 (this block's segment).
template <typename OffT, bool kAtomic>
__global__ __launch_bounds__(kRestoreBlock) void k_restore(SingleParams p, int lvl_arg) {
    constexpr int BLOCK = kRestoreBlock;
    __shared__ unsigned long long red[BLOCK / 64];
    __shared__ unsigned long long red_arcs[BLOCK / 64];
    __shared__ uint32_t tmp[BLOCK / 64];
    __shared__ uint32_t listed;  // next-frontier vertices of this block so far (the first kSmallSeg listed)
    __shared__ int32_t lids[kSmallSeg];  // the listed ids
    // Hub levels: the chunk's known visited bits, the bits its bins claim, and
    // the prefix of its bin regions' counts.
    __shared__ uint32_t known[BLOCK], claimed[BLOCK];
    __shared__ uint32_t rpre[kMaxBinGroups + 1];
    // Whether the run has ended, the level (step lvl_arg restores level
    // lvl_arg + the shift its expansion wrote) and (hybrid runs) the direction
    // of the level just expanded, read in one round (both parities).
    int binned = 0;
    const int dn = ld(&p.ctrl->done);
    const int sft = p.s_max > 0 ? ld(&p.ctrl->shift[(lvl_arg + 1) & 1]) : 0;
    int d2[2] = {0, 0};
    if (!kAtomic && p.hybrid) {
        d2[0] = ld(&p.ctrl->dir[0]);
        d2[1] = ld(&p.ctrl->dir[1]);
    }
    if (p.bin_k > 0) binned = ld(&p.ctrl->binned[lvl_arg & 1]);  // bins are off with small levels: no shift
    if (dn) return;
    const int lvl = lvl_arg + sft;
    const int dir_bu = d2[(lvl + 1) & 1];
    const int tid = threadIdx.x;
    if (tid == 0) listed = 0;
    __syncthreads();
    const int64_t G = gridDim.x, bid = blockIdx.x;
    const int next = lvl + 1;
    unsigned long long found = 0;
    unsigned long long list_arcs = 0;  // arcs of the rows this thread listed
    uint32_t seg_n = 0, seg_a = 0;  // running totals of this block's segment
    const int32_t first = p.seg_start[bid];
    // A bottom-up level wrote every changed word once, from its owner, with
    // exactly the new bits: no lost updates to put back.
    const bool exact_words = kAtomic || (p.hybrid && dir_bu != 0);
    for (int64_t c = bid; c * BLOCK < p.words; c += G) {
        const int64_t w = c * BLOCK + tid;
        const int lane = tid & 63;
        // ---- hub level: claim the heads binned for this chunk (bin c). This
        // block owns the chunk's words until it writes them below, so an LDS
        // bitmap claims every head exactly once; heads already visited before
        // the level (the snapshot) or claimed by the expansion's own path (the
        // current word) are skipped. Claims are recorded with device-scope
        // stores: the rebuild below reads the level array that way.
        uint32_t nb_w = 0;
        if (binned) {
            if (w < p.words) {
                known[tid] = ld(p.vis + w) | ld(p.vis_prev + w);
            } else {
                known[tid] = ~0u;
            }
            claimed[tid] = 0u;
            const int R = p.bin_groups;
            constexpr int PER = (kMaxBinGroups + BLOCK - 1) / BLOCK;
            uint32_t rc[PER], mine = 0;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int r = tid * PER + k;
                rc[k] = r < R ? ld(p.bin_cnt + (int64_t)r * p.bin_nb + c) : 0u;
                mine += rc[k];
            }
            uint32_t ex;
            const uint32_t total = block_excl_scan<BLOCK>(mine, ex, tmp);
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int r = tid * PER + k;
                if (r < R) rpre[r] = ex;
                ex += rc[k];
            }
            if (tid == 0) rpre[R] = total;
            __syncthreads();
            const unsigned long long* bins = reinterpret_cast<const unsigned long long*>(p.bin_e);
            constexpr int kBinUnroll = 4;
            for (uint32_t j0 = tid; j0 < total; j0 += BLOCK * kBinUnroll) {
                unsigned long long e[kBinUnroll];
                bool ok[kBinUnroll];
#pragma unroll
                for (int k = 0; k < kBinUnroll; ++k) {
                    const uint32_t j = j0 + k * BLOCK;
                    ok[k] = j < total;
                    int lo = 0, hi = R - 1;  // the region holding entry j: last with rpre <= j
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (rpre[mid] <= j) lo = mid; else hi = mid - 1;
                    }
                    const int64_t at = ((int64_t)c * R + lo) * p.bin_k + (j - rpre[lo]);
                    e[k] = ok[k] ? ld(bins + at) : 0ull;
                }
#pragma unroll
                for (int k = 0; k < kBinUnroll; ++k) {
                    if (!ok[k]) continue;
                    const int32_t v = (int32_t)(uint32_t)e[k];
                    const int32_t par = (int32_t)(uint32_t)(e[k] >> 32);
                    const uint32_t wl = ((uint32_t)v >> 5) - (uint32_t)(c * BLOCK);
                    const uint32_t b = 1u << (v & 31);
                    if (wl < (uint32_t)BLOCK && !(known[wl] & b) && !(atomicOr(&claimed[wl], b) & b))
                        record_st(p, v, next, par);
                }
            }
            __threadfence();
            __syncthreads();
            nb_w = claimed[tid];
        }
        uint32_t cur = 0, prev = 0, exact = 0, bm = 0;
        if (w < p.words) {
            cur = ld(p.vis + w);
            prev = ld(p.vis_prev + w);
            bm = p.bigmap[w];  // read-only graph data, read in the same round
        }
        // Words the expansion's own claims changed (racy in update mode 1),
        // and words with bin claims only (exact as they are).
        const bool racy = w < p.words && cur != prev;
        const bool touched = racy || nb_w != 0u;
        const uint32_t cur_mem = cur;  // the word as it stands in memory
        cur |= nb_w;
        if (exact_words) {
            exact = touched ? (cur & ~prev) : 0u;
        } else if (!__ballot(racy)) {
            exact = nb_w;
        } else {
            // A racing read-modify-write may have dropped bits of this level
            // (every writer read the word after the previous level's
            // restoration, so earlier bits survive; OR-ing the snapshot back
            // in guards them all the same), never added foreign ones, and
            // always leaves one of its bits set: the level array says exactly
            // who was discovered. Each half-wave reads one touched word's 32
            // levels; up to kRebuildPairs pairs of touched words per round,
            // all their level reads in flight together.
            exact = nb_w;  // words with bin claims only; the racy ones are rebuilt below
            uint64_t tm = __ballot(racy);
            const int64_t wave_w0 = c * BLOCK + (tid & ~63);
            while (tm) {
                int wa[kRebuildPairs], wb[kRebuildPairs], lvv[kRebuildPairs];
#pragma unroll
                for (int k = 0; k < kRebuildPairs; ++k) {
                    wa[k] = tm ? __builtin_ctzll(tm) : -1;
                    tm &= tm - 1;
                    wb[k] = tm ? __builtin_ctzll(tm) : -1;
                    tm &= tm - 1;
                }
#pragma unroll
                for (int k = 0; k < kRebuildPairs; ++k) {
                    const int src = lane < 32 ? wa[k] : wb[k];
                    const int64_t v = (wave_w0 + src) * 32 + (lane & 31);
                    const bool okl = src >= 0 && v < p.n;
                    const int x = ld(p.lv + (okl ? lv_at(p, v) : 0));
                    lvv[k] = okl ? x : -1;
                }
#pragma unroll
                for (int k = 0; k < kRebuildPairs; ++k) {
                    const uint64_t m = __ballot(lvv[k] == next);
                    if (lane == wa[k]) exact = (uint32_t)m;
                    if (lane == wb[k]) exact = (uint32_t)(m >> 32);
                }
            }
        }
        if (touched) {
            const uint32_t nv = prev | exact;
            if (cur_mem != nv) st(p.vis + w, nv);
            st(p.vis_prev + w, nv);
        }
        // Hot vertices of word w found this level: per hot bit position k,
        // one compact word per half-wavefront (slots w + k * span of its 32
        // words; span is a multiple of 32), written by its first lane only.
        if (p.hot_words > 0 && c * BLOCK < p.hot_span) {
            const int half = lane >> 5;
            const bool in = w < p.hot_span;
            for (int k = 0; k < (32 >> p.hot_shift); ++k) {
                const uint64_t hm = __ballot(in && ((exact >> (k << p.hot_shift)) & 1u));
                const uint32_t bits = (uint32_t)(hm >> (32 * half));
                const int64_t cw = (w >> 5) + (int64_t)k * (p.hot_span >> 5);
                if ((lane & 31) == 0 && bits) {
                    uint32_t* hw = p.hot_vis + cw;
                    st(hw, ld(hw) | bits);
                }
                if ((lane & 31) == 0 && in) st(p.hot_fr + cw, bits);
            }
        }
        if (w < p.words) {
            st(p.fr + w, exact);
            found += (unsigned long long)__popc(exact);
        }
        // List the block's next-frontier ids in LDS while there are few (for
        // the small-level path): one LDS atomic per wavefront, positions from
        // a wave scan.
        if (p.s_max > 0) {
            const int cnt = __popc(exact);
            const int inc = wave_incl_scan(cnt, lane);
            const int tot = __shfl(inc, 63, 64);
            uint32_t base = 0;
            if (lane == 63 && tot > 0) base = atomicAdd(&listed, (uint32_t)tot);
            base = (uint32_t)__shfl((int)base, 63, 64);
            uint32_t at = base + (uint32_t)(inc - cnt);
            for (uint32_t x = exact; x && at < (uint32_t)kSmallSeg; x &= x - 1, ++at)
                lids[at] = (int32_t)(w * 32 + __builtin_ctz(x));
        }
        // Append the next frontier's big rows of this chunk to the segment.
        const uint32_t big = exact & bm;
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
    // A block that listed its whole next frontier publishes the ids and the
    // arcs of their rows; one with more leaves the level to the grid (the
    // offset reads stay off the large levels, where nearly every block has more).
    const uint32_t nl = p.s_max > 0 ? listed : 0u;
    if (p.s_max > 0 && nl <= (uint32_t)kSmallSeg) {
        if (tid < (int)nl) {
            const int64_t v = lids[tid];
            st(p.sl + bid * kSmallSeg + tid, (int32_t)v);
            list_arcs = (unsigned long long)(load_off<OffT>(p.off, v + 1) - load_off<OffT>(p.off, v));
        }
        list_arcs = wave_sum(list_arcs);
        if ((tid & 63) == 0) red_arcs[tid >> 6] = list_arcs;
        __syncthreads();
    }
    if (tid == 0) {
        unsigned long long a = 0;
        for (int i = 0; i < BLOCK / 64; ++i) a += red[i];
        if (a) {
            atomicAdd(stripe(p.ctrl, next & 1, (int)(bid % kStripes)), a);
            atomicAdd(p.reached_slot + bid, a);
        }
        st(p.seg_cnt + bid, seg_n);
        st(p.seg_arcs + bid, seg_a);
        if (seg_a) atomicAdd(&p.ctrl->bigarcs[next & 1][(bid % kStripes) * kStripeStride], (unsigned long long)seg_a);
        if (p.s_max > 0) {
            st(p.sl_cnt + bid, (int32_t)nl);
            // Only blocks that listed all their ids count them (so the sum
            // equals the level's count exactly when every block did).
            if (nl > 0 && nl <= (uint32_t)kSmallSeg) {
                unsigned long long sa = 0;
                for (int i = 0; i < BLOCK / 64; ++i) sa += red_arcs[i];
                unsigned long long* sp = stripe(p.ctrl, next & 1, (int)(bid % kStripes));
                atomicAdd(sp + 1, sa);
                atomicAdd(sp + 2, (unsigned long long)nl);
            }
        }
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

// Reached vertices and the sum of their degrees, from a level array.
template <typename OffT>
__global__ void k_stats_levels(const int32_t* lv, const OffT* off, int64_t n, Ctrl* c) {
    unsigned long long r = 0, a = 0;
    const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gsize)
        if (lv[v] >= 0) {
            ++r;
            a += (unsigned long long)((int64_t)off[v + 1] - (int64_t)off[v]);
        }
    r = wave_sum(r);
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) {
        if (r) atomicAdd(&c->reached, r);
        if (a) atomicAdd(&c->arcs, a);
    }
}

// Symmetry check: the multiset of arcs and the multiset of reversed arcs have
// the same sum of a 64-bit hash; one wavefront per row.
__device__ __forceinline__ unsigned long long arc_hash(uint32_t a, uint32_t b) {
    unsigned long long z = ((unsigned long long)a << 32 | b) + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

template <typename OffT>
__global__ void k_symmetry(const OffT* off, const int32_t* col, int64_t n, unsigned long long* sums) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long fwd = 0, rev = 0;
    for (int64_t u = wave; u < n; u += waves) {
        const int64_t b = (int64_t)off[u], e = (int64_t)off[u + 1];
        for (int64_t j = b + lane; j < e; j += 64) {
            const uint32_t v = (uint32_t)col[j];
            fwd += arc_hash((uint32_t)u, v);
            rev += arc_hash(v, (uint32_t)u);
        }
    }
    fwd = wave_sum(fwd);
    rev = wave_sum(rev);
    if (lane == 0) {
        atomicAdd(sums, fwd);
        atomicAdd(sums + 1, rev);
    }
}

// Columns of the degree-ordered copy: new row x is caller row new2old[x] with
// every neighbour renamed; one wavefront per row, arcs in their original order.
template <typename OffT>
__global__ void k_relabel_cols(const OffT* off, const int32_t* col, const int64_t* noff, const int32_t* new2old,
                               const int32_t* old2new, int32_t* ncol, int64_t n, int32_t hot_span,
                               int32_t hot_shift, int32_t big_threshold, int32_t blk_shift, int32_t nblk,
                               uint32_t* bseg) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t x = wave; x < n; x += waves) {
        const int64_t u = new2old[x];
        const int64_t b = (int64_t)off[u], d = (int64_t)off[u + 1] - b, nb = noff[x];
        if (nblk > 0 && d > big_threshold) {
            // Row above T2: columns grouped by destination block (stable),
            // lane k < nblk counting block k; then the first arc of every
            // block and the degree go to the row's entry (its hot rank).
            uint32_t cnt = 0;
            for (int64_t j0 = 0; j0 < d; j0 += 64) {
                const int64_t j = j0 + lane;
                const int blk = j < d ? (int)((uint32_t)old2new[col[b + j]] >> blk_shift) : -1;
                uint64_t todo = __ballot(blk >= 0);
                while (todo) {
                    const int k = __shfl(blk, __builtin_ctzll(todo), 64);
                    const uint64_t m = __ballot(blk == k);
                    if (lane == k) cnt += (uint32_t)__popcll(m);
                    todo &= ~m;
                }
            }
            const int excl = wave_incl_scan((int)cnt, lane) - (int)cnt;
            uint32_t rank = 0;
            const bool hot = hot_slot((uint32_t)x, (uint32_t)hot_span, (uint32_t)hot_shift, rank);
            if (hot && lane < nblk) bseg[(size_t)rank * (nblk + 1) + lane] = (uint32_t)excl;
            if (hot && lane == 0) bseg[(size_t)rank * (nblk + 1) + nblk] = (uint32_t)d;  // nblk may be 64
            int cursor = excl;  // lane k: next slot of block k
            for (int64_t j0 = 0; j0 < d; j0 += 64) {
                const int64_t j = j0 + lane;
                const int32_t v = j < d ? old2new[col[b + j]] : -1;
                const int blk = v >= 0 ? (int)((uint32_t)v >> blk_shift) : -1;
                uint64_t todo = __ballot(blk >= 0);
                while (todo) {
                    const int k = __shfl(blk, __builtin_ctzll(todo), 64);
                    const uint64_t m = __ballot(blk == k);
                    const int at = __shfl(cursor, k, 64);
                    if (blk == k) ncol[nb + at + rank_in(m)] = v;
                    if (lane == k) cursor += __popcll(m);
                    todo &= ~m;
                }
            }
            continue;
        }
        if (d <= 64) {
            // Short row: one sort across the wavefront. Hot neighbours first by
            // rank (highest degree first), then the others in arc order.
            const int32_t v = lane < d ? old2new[col[b + lane]] : -1;
            uint32_t rank = 0;
            const bool is_hot = v >= 0 && hot_slot((uint32_t)v, (uint32_t)hot_span, (uint32_t)hot_shift, rank);
            unsigned long long key = v < 0 ? ~0ull
                                           : (is_hot ? (unsigned long long)rank
                                                     : (1ull << 40) | (unsigned long long)lane);
            int32_t val = v;
            for (int k = 2; k <= 64; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    const unsigned long long ok_ = ((unsigned long long)__shfl_xor((int)(key >> 32), j, 64) << 32) |
                                                   (uint32_t)__shfl_xor((int)(uint32_t)key, j, 64);
                    const int32_t ov = __shfl_xor(val, j, 64);
                    const bool up = (lane & k) == 0;          // this pair sorts ascending
                    const bool low = (lane & j) == 0;         // this lane keeps the smaller key
                    const bool take = (low == up) ? ok_ < key : ok_ > key;
                    if (take) {
                        key = ok_;
                        val = ov;
                    }
                }
            }
            if (lane < d) ncol[nb + lane] = val;
            continue;
        }
        // Long row: two stable passes, hot neighbours first, then the rest.
        int64_t at = 0;
        for (int pass = 0; pass < 2; ++pass) {
            for (int64_t j0 = 0; j0 < d; j0 += 64) {
                const int64_t j = j0 + lane;
                const int32_t v = j < d ? old2new[col[b + j]] : -1;
                uint32_t rank = 0;
                const bool is_hot = v >= 0 && hot_slot((uint32_t)v, (uint32_t)hot_span, (uint32_t)hot_shift, rank);
                const bool take = v >= 0 && (pass == 0 ? is_hot : !is_hot);
                const uint64_t m = __ballot(take);
                if (take) ncol[nb + at + rank_in(m)] = v;
                at += __popcll(m);
            }
        }
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
int occupancy_of(K kernel, int block, size_t dyn_lds = 0) {
    int occ = 0;
    hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, block, dyn_lds), "occupancy query");
    return occ;
}

struct Grids {
    int expand;
    int restore;
};

// Dynamic LDS available to one expansion workgroup next to its static LDS.
template <int BLOCK>
int lds_dynamic_cap() {
    constexpr int kLdsPerCu = 160 * 1024;
    const int left = kLdsPerCu - (int)sizeof(ExpandShared<BLOCK>) - 1024;  // margin for compiler temporaries
    return std::min(left, kMaxHotWords * 4);
}


template <typename OffT, int BLOCK, bool kAtomic>
Grids grids_for(bfs_graph* g, const bfs_tunables& t, int64_t nslots, int lds_words) {
    // Dynamic LDS (the hot snapshot) beyond the default limit must be allowed
    // once: up to what fits beside the static LDS in the 160 KiB of a CU.
    const int cap = lds_dynamic_cap<BLOCK>();
    static const bool lds_ok = hipFuncSetAttribute(reinterpret_cast<const void*>(k_expand<OffT, BLOCK, kAtomic>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, cap) == hipSuccess;
    if (!lds_ok) fail(BFS_E_DEVICE, "cannot enable dynamic LDS for the expansion kernel");
    if (lds_words * 4 > cap) fail(BFS_E_INVALID_ARG, "LDS bitmap does not fit beside this workgroup size");
    const int occ = occupancy_of(k_expand<OffT, BLOCK, kAtomic>, BLOCK, (size_t)lds_words * 4);
    // On gfx950 one workgroup per CU fewer than the occupancy query reports is
    // resident at once (measured: with the reported count, one workgroup per CU
    // starts only when another finishes); a grid that fits keeps every
    // workgroup's share in the first wave of the dispatch.
    const int fit = occ > 1 ? occ - 1 : 1;
    const int bpc = t.blocks_per_cu > 0 && t.blocks_per_cu < fit ? t.blocks_per_cu : fit;
    int64_t ge = (int64_t)bpc * g->cu_count;
    ge = std::max<int64_t>(1, std::min(ge, nslots));
    if (g->restore_grid < 1 || g->restore_grid > kMaxRestoreGrid || g->restore_grid > nslots)
        fail(BFS_E_INTERNAL, "restore grid out of range");
    return Grids{(int)ge, g->restore_grid};
}

template <typename OffT, int BLOCK, bool kAtomic>
void launch_typed(bfs_graph* g, const bfs_tunables& t, Workspace* w, SingleParams& p, hipStream_t s,
                  hipEvent_t stop) {
    // Dynamic LDS: the largest of the visited copy, a destination block, the
    // bin counters and the small-level lists (5 words an entry).
    const int lds_words = std::max<int>(std::max<int>(std::max<int>(std::max<int>(p.hot_words, p.full_words),
                                                                    p.bseg ? 1 << (p.blk_shift - 5) : 0),
                                                      p.bin_e ? p.bin_nb : 0),
                                        p.s_max > 0 ? 5 * kSmallMax : 0);
    const Grids gr = grids_for<OffT, BLOCK, kAtomic>(g, t, w->nslots, lds_words);
    // Bins: one region per (bin, expansion workgroup), as many entries as the
    // workspace's bin storage gives each; too few and the bins stay off.
    if (p.bin_e && gr.expand <= kMaxBinGroups) {
        const int64_t k = w->bin_cap / ((int64_t)p.bin_nb * gr.expand);
        if (k >= 8) {
            p.bin_k = (int32_t)std::min<int64_t>(k, 1 << 20);
            p.bin_groups = gr.expand;
        }
    }
    // Block-by-block expansion pays off once every workgroup has a few
    // hundred arcs of the big rows to walk.
    p.blk_min_arcs = (int64_t)gr.expand * 256;
    const int init_grid = (int)std::min<int64_t>(std::max<int64_t>(p.n / 4, p.words) / BLOCK + 1, 4096);
    k_init<OffT, BLOCK><<<init_grid, BLOCK, 0, s>>>(p, (int)w->nslots);
    BFS_HIP(hipGetLastError());
    // Steps are enqueued in chunks; between chunks the host reads the done
    // flag. A step is one expansion and one restoration; step s works on level
    // s plus the levels earlier small-level loops ran beyond their own (kept
    // in the control block). The first chunk covers as many steps as the
    // previous run on this workspace used (runs from other roots of one graph
    // have similar shapes), so most runs end inside it.
    // When the previous run's step count says this chunk ends the run, the
    // output pass and the stop event go in before the host waits, so the
    // host's wake-up is not inside the timed span; if the run goes on, a later
    // chunk repeats both.
    const int64_t expect = w->last_launches;  // 0: unknown
    int64_t steps = 0;
    int chunk = std::max(4, std::min(64, w->last_launches + 1));
    bool finished_early = false;
    auto finish = [&] {
        if (p.new2old) {
            const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((p.n + 255) / 256, (int64_t)g->cu_count * 16));
            k_out<<<blocks, 256, 0, s>>>(reinterpret_cast<const unsigned long long*>(p.lv), p.old2new, p.out_lv,
                                         p.out_pa, p.n);
            BFS_HIP(hipGetLastError());
        }
        if (stop) BFS_HIP(hipEventRecord(stop, s));
    };
    while (true) {
        for (int i = 0; i < chunk; ++i) {
            const int step = (int)(steps + i);
            k_expand<OffT, BLOCK, kAtomic><<<gr.expand, BLOCK, (size_t)lds_words * 4, s>>>(p, step);
            k_restore<OffT, kAtomic><<<gr.restore, kRestoreBlock, 0, s>>>(p, step);
        }
        BFS_HIP(hipGetLastError());
        steps += chunk;
        finished_early = expect > 0 && steps >= expect;
        if (finished_early) finish();
        static_assert(offsetof(Ctrl, steps) == offsetof(Ctrl, done) + 3 * sizeof(int), "done .. steps");
        BFS_HIP(hipMemcpyAsync(&w->host_ctrl->done, &p.ctrl->done, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
        BFS_HIP(hipStreamSynchronize(s));
        if (w->host_ctrl->done || steps > p.n + 1) break;
        chunk = chunk < 64 ? chunk * 2 : 64;
    }
    // The step that found the frontier empty was the last one with work.
    if (w->host_ctrl->done) w->last_launches = w->host_ctrl->steps;
    if (!finished_early) finish();
}

}  // namespace

int64_t lds_visited_words_max(int block) {
    const int cap = block == 1024 ? lds_dynamic_cap<1024>() : block == 512 ? lds_dynamic_cap<512>()
                                                                           : lds_dynamic_cap<256>();
    return cap / 4 / 64 * 64;
}

void launch_single(bfs_graph* g, const bfs_tunables& t, Workspace* w, int32_t root, int32_t* levels,
                   int32_t* parents, hipStream_t s, bool hybrid, hipEvent_t stop) {
    // Host-side checks of what the kernels assume about their buffers.
    if (root < 0 || root >= g->n) fail(BFS_E_ROOT_RANGE, "root out of range");
    if (w->words * 32 < g->n || w->words % 64 != 0) fail(BFS_E_INTERNAL, "workspace bitmaps too small");
    if (!levels || !parents) fail(BFS_E_INVALID_ARG, "NULL output");
    // The degree-ordered copy with its LDS hot bitmap, or the caller's order.
    const int32_t want_hot = hot_count(g, t);
    const HotLayout* h = want_hot > 0 ? g->hot.get() : nullptr;
    if (want_hot > 0 && (!h || h->hot != want_hot)) fail(BFS_E_INTERNAL, "degree-ordered copy out of date");
    if (h && (!w->run_rec || (reinterpret_cast<uintptr_t>(w->run_rec) & 15) != 0))
        fail(BFS_E_INTERNAL, "workspace lacks the run records of the copy");
    const BigTable& bt = h ? h->big : g->big;
    if (bt.threshold != t.wave_max_degree) fail(BFS_E_INTERNAL, "big-row table out of date");
    SingleParams p{};
    p.off = h ? static_cast<const void*>(h->d_off) : g->d_off;
    p.col = h ? h->d_col : g->d_col;
    p.n = (int32_t)g->n;
    p.root = h ? h->old2new[(size_t)root] : root;
    p.root_out = root;
    p.words = w->words;
    p.lv = h ? w->run_rec : levels;
    p.out_lv = levels;
    p.out_pa = parents;
    p.new2old = h ? h->d_new2old : nullptr;
    p.old2new = h ? h->d_old2new : nullptr;
    p.vis = w->vis;
    p.vis_prev = w->vis_prev;
    p.fr = w->fr;
    p.ctrl = w->ctrl;
    p.arcs_slot = w->slots;
    p.reached_slot = w->slots + w->nslots;
    p.bigmap = bt.d_bigmap;
    p.nzmap = bt.d_nzmap;
    p.bl_u = w->bl_u;
    p.bl_pre = w->bl_pre;
    p.seg_cnt = w->seg_cnt;
    p.seg_arcs = w->seg_arcs;
    p.seg_start = bt.d_seg_start;
    p.restore_grid = g->restore_grid;
    p.t1 = t.small_max_degree;
    p.min_share = t.chunk_arcs > 0 ? t.chunk_arcs : 1024;
    // Destination blocks of the copy's rows above T2 (built for this T2 and
    // block size, and fitting the LDS bitmap of the expansion workgroup).
    const bool blocked = h && h->nblk > 0 && h->d_bseg && h->blk_req == t.block_vertices &&
                         ((int64_t)1 << (h->blk_shift - 5)) <= lds_visited_words_max(t.block_size);
    p.bseg = blocked ? h->d_bseg : nullptr;
    p.bseg_rows = blocked ? h->big.num_big : 0;
    p.nblk = blocked ? h->nblk : 0;
    p.blk_shift = blocked ? h->blk_shift : 0;
    p.blk_min_arcs = 0;  // set with the grid
    // Destination bins of hub levels (entries per region set with the grid).
    const int64_t nbins = (w->words + kRestoreBlock - 1) / kRestoreBlock;
    const bool bins = t.hub_bins > 0 && w->bin_e && w->bin_cnt && t.sparse_frontier <= 0 &&
                      nbins <= lds_visited_words_max(t.block_size) && nbins * kMaxBinGroups <= w->bin_cnt_cap;
    p.bin_e = bins ? w->bin_e : nullptr;
    p.bin_cnt = bins ? w->bin_cnt : nullptr;
    p.bin_nb = bins ? (int32_t)nbins : 0;
    p.bin_k = 0;
    p.bin_groups = 0;
    p.hot_words = h ? h->hot / 32 : 0;
    p.hot_shift = h ? h->shift : 5;
    p.hot_span = h ? h->span : 0;
    p.hot_vis = w->hot_vis;
    p.hot_fr = w->hot_fr;
    p.hot_min_frontier = std::max<int64_t>(4096, g->n / 256);
    p.full_words = (int32_t)lds_visited_words(g, t);
    if (p.full_words % 64 != 0 || p.full_words > w->words) fail(BFS_E_INTERNAL, "LDS visited words out of range");
    if ((int64_t)p.hot_words * 32 > w->words * 2 || p.hot_words % 2 != 0 || p.hot_words > w->hot_capacity)
        fail(BFS_E_INTERNAL, "hot bitmap larger than its buffer");
    if (h && (h->hot % 64 != 0 || (h->shift != 5 && h->shift != 4) || h->span != (h->hot / 32) << h->shift ||
              h->span % 32 != 0 || (int64_t)h->span * 32 > g->n))
        fail(BFS_E_INTERNAL, "hot layout out of range");
    if (w->big_capacity < bt.num_big) fail(BFS_E_INTERNAL, "big-row list too small");
    if (hybrid && !g->symmetric) fail(BFS_E_INVALID_ARG, "bottom-up levels need a graph loaded as symmetric");
    p.nnz = g->nnz;
    p.hybrid = hybrid ? 1 : 0;
    p.sl = w->sl;
    p.sl_cnt = w->sl_cnt;
    p.s_max = t.sparse_frontier > 0 ? std::min(t.sparse_frontier, kSmallMax) : 0;
    p.s_arcs = (int64_t)p.s_max * 4;
    if (!p.sl || !p.sl_cnt || g->restore_grid > kMaxRestoreGrid) fail(BFS_E_INTERNAL, "small-level lists out of range");
    const bool off32 = !h && g->off32;
    const bool atomic = t.update_mode == 2;
#define BFS_LAUNCH(OFFT, BS)                                         \
    do {                                                             \
        if (atomic)                                                  \
            launch_typed<OFFT, BS, true>(g, t, w, p, s, stop);       \
        else                                                         \
            launch_typed<OFFT, BS, false>(g, t, w, p, s, stop);      \
    } while (0)
    if (off32) {
        if (t.block_size == 1024)
            BFS_LAUNCH(int32_t, 1024);
        else if (t.block_size == 512)
            BFS_LAUNCH(int32_t, 512);
        else
            BFS_LAUNCH(int32_t, 256);
    } else {
        if (t.block_size == 1024)
            BFS_LAUNCH(int64_t, 1024);
        else if (t.block_size == 512)
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

void launch_single_stats_from_levels(bfs_graph* g, const bfs_tunables& t, Workspace* w, const int32_t* levels,
                                     hipStream_t s) {
    (void)t;  // the caller's levels are complete on either layout
    if (!levels) fail(BFS_E_INTERNAL, "no level array for the stats");
    BFS_HIP(hipMemsetAsync(&w->ctrl->reached, 0, 2 * sizeof(unsigned long long), s));
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((g->n + 255) / 256, (int64_t)g->cu_count * 8));
    if (g->off32)
        k_stats_levels<int32_t><<<blocks, 256, 0, s>>>(levels, static_cast<const int32_t*>(g->d_off), g->n, w->ctrl);
    else
        k_stats_levels<int64_t><<<blocks, 256, 0, s>>>(levels, static_cast<const int64_t*>(g->d_off), g->n, w->ctrl);
    BFS_HIP(hipGetLastError());
}

bool csr_is_symmetric(const bfs_graph* g) {
    unsigned long long* d = nullptr;
    unsigned long long h[2] = {0, 0};
    BFS_HIP(hipMalloc(&d, 2 * sizeof(unsigned long long)));
    try {
        BFS_HIP(hipMemset(d, 0, 2 * sizeof(unsigned long long)));
        const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((g->n + 3) / 4, (int64_t)g->cu_count * 32));
        if (g->off32)
            k_symmetry<int32_t><<<blocks, 256>>>(static_cast<const int32_t*>(g->d_off), g->d_col, g->n, d);
        else
            k_symmetry<int64_t><<<blocks, 256>>>(static_cast<const int64_t*>(g->d_off), g->d_col, g->n, d);
        BFS_HIP(hipGetLastError());
        BFS_HIP(hipMemcpy(h, d, sizeof(h), hipMemcpyDeviceToHost));
    } catch (...) {
        (void)hipFree(d);
        throw;
    }
    (void)hipFree(d);
    return h[0] == h[1];
}

void launch_relabel_cols(const bfs_graph* g, const int64_t* d_noff, const int32_t* d_new2old,
                         const int32_t* d_old2new, int32_t* d_ncol, int32_t hot_span, int32_t hot_shift,
                         int32_t big_threshold, int32_t blk_shift, int32_t nblk, uint32_t* d_bseg) {
    if (nblk > kMaxBlocks || (nblk > 0 && (!d_bseg || blk_shift < 11 || blk_shift > 20)))
        fail(BFS_E_INTERNAL, "destination blocks out of range");
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((g->n + 3) / 4, (int64_t)g->cu_count * 32));
    if (g->off32)
        k_relabel_cols<int32_t><<<blocks, 256>>>(static_cast<const int32_t*>(g->d_off), g->d_col, d_noff, d_new2old,
                                                 d_old2new, d_ncol, g->n, hot_span, hot_shift, big_threshold,
                                                 blk_shift, nblk, d_bseg);
    else
        k_relabel_cols<int64_t><<<blocks, 256>>>(static_cast<const int64_t*>(g->d_off), g->d_col, d_noff, d_new2old,
                                                 d_old2new, d_ncol, g->n, hot_span, hot_shift, big_threshold,
                                                 blk_shift, nblk, d_bseg);
    BFS_HIP(hipGetLastError());
}

void launch_fill_i32(int32_t* ptr, int64_t count, int32_t value, hipStream_t s) {
    if (count <= 0) return;
    const int blocks = (int)(count / 1024 + 1 < 4096 ? count / 1024 + 1 : 4096);
    k_fill_i32<<<blocks, 256, 0, s>>>(ptr, count, value);
    BFS_HIP(hipGetLastError());
}

}  // namespace bfs
