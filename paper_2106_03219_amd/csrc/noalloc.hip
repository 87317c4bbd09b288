// noalloc.hip -- omprt_reduce_noalloc: the plain reduction (and its
// exact-map variant) with its cross-team state in a fixed device array
// instead of a per-stream workspace, for callers that cannot allocate.
//
// The array, `scratch`, holds the same layout as a workspace: a 256-byte
// header (election counter, launch epoch, status bits) and one 32-byte
// tagged slot per team, for up to kNoAllocTeams teams.  It starts zeroed
// (static storage) and keeps the workspace invariants from call to call:
// the election leaves the counter at 0, the finisher advances the epoch,
// and slot tags are odd, so a zeroed slot never matches.  Every call on a
// device uses that device's one copy, so calls on one device must not
// overlap (two streams at once would mix their counters and slots).
//
// In host code the array's name is only a stand-in for the symbol: its
// device address comes from hipGetSymbolAddress, once per device with that
// device current, and that address is what the kernels receive.
#include <mutex>

#include "launch.h"
#include "runtime.h"

namespace omprt {

constexpr int kNoAllocTeams = 4096;
constexpr size_t kNoAllocBytes = 256 + (size_t)kNoAllocTeams * kSlotBytes;   // 128 KiB + 256 B

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes] = {};

constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[kNoAllocMaxDevices] = {};

// Device address of the current device's scratch (looked up once per device).
static omprt_status noalloc_scratch(int dev, void** out) {
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(OMPRT_ERR_UNSUPPORTED, "device %d beyond %d", dev, kNoAllocMaxDevices);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(OMPRT_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return OMPRT_OK;
}

}  // namespace omprt

using namespace omprt;

extern "C" omprt_status omprt_reduce_noalloc(const void* d_in, int64_t n, int32_t dtype,
                                             int32_t op, void* d_x, const omprt_config* cfg,
                                             void* hip_stream) {
    if (dtype < 0 || dtype >= DT_COUNT_ABI) return fail(OMPRT_ERR_UNSUPPORTED, "dtype %d", dtype);
    if (!op_defined(dtype, op)) return fail(OMPRT_ERR_UNSUPPORTED, "op %d on dtype %d", op, dtype);
    if (n < 0 || n > ((int64_t)1 << 50))
        return fail(OMPRT_ERR_INVALID, "n = %lld outside 0..2^50", (long long)n);
    if (!d_x) return fail(OMPRT_ERR_INVALID, "x is NULL");
    if (n > 0 && !d_in) return fail(OMPRT_ERR_INVALID, "input is NULL with n > 0");
    if (reinterpret_cast<uintptr_t>(d_in) % (uintptr_t)dtype_bytes(dtype) != 0)
        return fail(OMPRT_ERR_INVALID, "input is not %d-byte aligned", dtype_bytes(dtype));
    if (reinterpret_cast<uintptr_t>(d_x) % (uintptr_t)out_bytes(dtype, op) != 0)
        return fail(OMPRT_ERR_INVALID, "x is not %d-byte aligned", out_bytes(dtype, op));
    const bool exact = cfg && (cfg->flags & OMPRT_CFG_EXACT_THREAD_MAP);
    if (exact && op > OMPRT_MIN)
        return fail(OMPRT_ERR_UNSUPPORTED, "EXACT_THREAD_MAP takes sum, max and min");
    LaunchCfg lc;
    if (omprt_status st = resolve_config(n, dtype, op, 0, -1, cfg, &lc, nullptr)) return st;
    if (lc.teams > kNoAllocTeams)
        return fail(OMPRT_ERR_INVALID,
                    "%d teams: the fixed cross-team scratch holds %d (use omprt_reduce)",
                    lc.teams, kNoAllocTeams);
    if (n == 0) return OMPRT_OK;
    int dev = 0;
    OMPRT_HIP(hipGetDevice(&dev));
    void* base = nullptr;
    if (omprt_status st = noalloc_scratch(dev, &base)) return st;
    uint32_t* words = static_cast<uint32_t*>(base);
    const CrossTeamArgs ct{static_cast<char*>(base) + 256, words, words + 32, words + 48};
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const hipError_t e =
        exact ? launch_reduce_exact(dtype, op, d_in, n, d_x, lc.teams, lc.threads, ct, stream)
              : launch_reduce(dtype, op, lc.vec, lc.unroll, d_in, n, d_x, lc.teams, lc.threads, ct,
                              stream);
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "reduce launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}
