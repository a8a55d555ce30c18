// Memory-system ceilings of the GPU the BFS kernels run on, measured with
// small kernels of the same access shapes: a streaming read, a copy, random
// 4-byte gathers from tables of a chosen size, random device-scope atomicOr
// without a returned value, and back-to-back empty launches. Each call times
// `iters` launches with HIP events on the null stream and returns the mean
// milliseconds per launch. Buffers belong to the caller (device pointers).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kBlock = 256;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte load or store

// SplitMix64 finaliser (Steele, Lea and Flood): a counter-based hash used to
// draw uniform table positions without an index array.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBlock) void k_read(const u32x4* src, int64_t n16, uint32_t* sink) {
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += stride) {
        const u32x4 v = __builtin_nontemporal_load(src + i);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;  // keeps the loads; practically never stores
}

__global__ __launch_bounds__(kBlock) void k_copy(u32x4* dst, const u32x4* src, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Each thread issues 8 independent gathers per round, the shape of the
// expansion kernels' visited probes.
__global__ __launch_bounds__(kBlock) void k_gather(const uint32_t* table, uint64_t words, int64_t count,
                                                   uint64_t seed, uint32_t* sink) {
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock * 8;
    for (int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 8; i < count; i += stride) {
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = table[mix64(seed + (uint64_t)(i + k)) & (words - 1)];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc ^= v[k];
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

__global__ __launch_bounds__(kBlock) void k_atomic_or(uint32_t* table, uint64_t words, int64_t count, uint64_t seed) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
        const uint64_t h = mix64(seed + (uint64_t)i);
        atomicOr(table + (h & (words - 1)), 1u << (h >> 59));
    }
}

__global__ void k_empty() {}

int grid_for(int64_t items) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const int64_t want = (items + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)cus * 16;
    return (int)(want < 1 ? 1 : want < cap ? want : cap);
}

template <typename L>
int timed(int iters, float* ms, L&& launch) {
    if (iters < 1 || !ms) return -1;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -5;
    launch();  // warm-up
    int rc = hipEventRecord(a, nullptr) == hipSuccess ? 0 : -5;
    for (int i = 0; i < iters && rc == 0; ++i) launch();
    if (rc == 0 && hipGetLastError() != hipSuccess) rc = -5;
    if (rc == 0 && hipEventRecord(b, nullptr) != hipSuccess) rc = -5;
    if (rc == 0 && hipEventSynchronize(b) != hipSuccess) rc = -5;
    float t = 0.f;
    if (rc == 0 && hipEventElapsedTime(&t, a, b) != hipSuccess) rc = -5;
    *ms = t / (float)iters;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return rc;
}

}  // namespace

extern "C" {

// Streaming read of `bytes` (a multiple of 16) from `src`; `sink` is one word.
int ceil_read(const void* src, int64_t bytes, uint32_t* sink, int iters, float* ms) {
    if (!src || !sink || bytes < 16 || bytes % 16) return -1;
    const int64_t n16 = bytes / 16;
    const int g = grid_for(n16);
    return timed(iters, ms, [&] { k_read<<<g, kBlock>>>(static_cast<const u32x4*>(src), n16, sink); });
}

// Copy of `bytes` (a multiple of 16) from `src` to `dst`.
int ceil_copy(void* dst, const void* src, int64_t bytes, int iters, float* ms) {
    if (!src || !dst || bytes < 16 || bytes % 16) return -1;
    const int64_t n16 = bytes / 16;
    const int g = grid_for(n16);
    return timed(iters, ms,
                 [&] { k_copy<<<g, kBlock>>>(static_cast<u32x4*>(dst), static_cast<const u32x4*>(src), n16); });
}

// `count` (a multiple of 8) random 4-byte reads from a table of `words` words
// (a power of two, so a position is a mask of the hash, not a division).
int ceil_gather(const uint32_t* table, int64_t words, int64_t count, uint32_t* sink, int iters, float* ms) {
    if (!table || !sink || words < 1 || (words & (words - 1)) || count < 8 || count % 8) return -1;
    const int g = grid_for(count / 8);
    uint64_t seed = 1;
    return timed(iters, ms, [&] { k_gather<<<g, kBlock>>>(table, (uint64_t)words, count, seed++, sink); });
}

// `count` random device-scope atomicOr (no returned value) into a table of
// `words` words (a power of two).
int ceil_atomic_or(uint32_t* table, int64_t words, int64_t count, int iters, float* ms) {
    if (!table || words < 1 || (words & (words - 1)) || count < 1) return -1;
    const int g = grid_for(count);
    uint64_t seed = 1;
    return timed(iters, ms, [&] { k_atomic_or<<<g, kBlock>>>(table, (uint64_t)words, count, seed++); });
}

// Back-to-back launches of an empty one-workgroup kernel.
int ceil_empty(int iters, float* ms) {
    return timed(iters, ms, [&] { k_empty<<<1, 64>>>(); });
}

}  // extern "C"
