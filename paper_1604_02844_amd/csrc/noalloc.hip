// Single-root BFS that allocates nothing: the kernels and launch sequence of
// bfs_run, with every scratch buffer of the run (bitmaps, control block,
// per-block sums, big-row and small-frontier lists, hot bitmaps, run records)
// carved from one statically sized device array instead of a pooled
// workspace. For callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bfs_internal.h"

namespace bfs {
namespace {

constexpr size_t kScratchBytes = (size_t)BFS_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");
constexpr int kMaxDevices = 64;

// One copy per device, resident from module load until the process ends. In
// host code this name is a stand-in, not a device address: kernels and copies
// get the address hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
    std::mutex mu;          // one call at a time per device: they share the array
    void* ptr = nullptr;    // device address of `scratch` on this device
    Ctrl host{};            // host mirror of the control block (done flag between chunks)
    int last_launches = 0;  // level steps of the previous call (first chunk size)
};
DeviceScratch g_dev[kMaxDevices];

// Held for the run: a graph's tunables and tables cannot change meanwhile
// (bfs_graph_set_tunables reports BFS_E_BUSY while a run is in progress).
struct RunHold {
    bfs_graph* g;
    explicit RunHold(bfs_graph* gr) : g(gr) {}
    ~RunHold() {
        std::lock_guard<std::mutex> lk(g->mu);
        --g->ws_out;
    }
};

}  // namespace

void run_noalloc(bfs_graph* g, int32_t root, int32_t* levels, int32_t* parents, hipStream_t s, bool hybrid) {
    if (g->device < 0 || g->device >= kMaxDevices) fail(BFS_E_INVALID_ARG, "device index beyond the scratch table");
    DeviceScratch& d = g_dev[g->device];
    std::lock_guard<std::mutex> dev_lock(d.mu);
    if (!d.ptr) {
        // Set-up, once per device, with that device current (the caller's
        // DeviceScope): the array's address on this device.
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) hip_check(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        d.ptr = ptr;
    }
    bfs_tunables t{};
    Workspace w{};
    {
        std::lock_guard<std::mutex> lk(g->mu);
        t = resolve_tunables(g, g->tun);
        if (ws_layout(g, &w, nullptr, false) > kScratchBytes)
            fail(BFS_E_NO_MEMORY, "the run needs more scratch than the static array holds");
        ++g->ws_out;
    }
    RunHold hold(g);
    ws_layout(g, &w, static_cast<char*>(d.ptr), false);
    w.host_ctrl = &d.host;
    w.last_launches = d.last_launches;
    // The array keeps the previous call's contents: the control block starts
    // at zero (k_init resets everything else the run reads). A fill kernel,
    // not a memset, so that the sequence holds only kernel launches.
    static_assert(sizeof(Ctrl) % 4 == 0, "Ctrl is filled in 32-bit words");
    launch_fill_i32(reinterpret_cast<int32_t*>(w.ctrl), (int64_t)(sizeof(Ctrl) / 4), 0, s);
    launch_single(g, t, &w, root, levels, parents, s, hybrid, nullptr);
    // The output pass may still be queued: the call returns when the run is
    // complete, so the next call may reuse the array.
    BFS_HIP(hipStreamSynchronize(s));
    d.last_launches = w.last_launches;
}

}  // namespace bfs
