// histogram.hip -- reduction(+: hist[0:bins]) over a loop whose iteration i
// does hist[key[i]] += 1: an array-section reduction whose list item is
// chosen by the data.  Each team takes a team-shared copy of (a range of)
// the histogram with team_alloc (in LDS when it fits, else in its slice of
// a global pool), counts its balanced block of keys into it with atomic
// adds, and adds the non-zero bins of its copy into hist.  Past the LDS
// ranges the default is no copy at all: atomic adds on hist.  Counts wrap modulo 2^32; keys
// outside [0, bins) are not counted and set bit 3 (value 4) of the stream's
// workspace status.
#include <algorithm>
#include <map>
#include <mutex>

#include "device.h"
#include "runtime.h"
#include "shared_alloc.h"

namespace omprt {

typedef __attribute__((address_space(3))) uint32_t lds_u32;

// The team copy lives in LDS (LdsCopy, ds atomics) or in the team's slice of
// the global pool (GlobalCopy, atomics performed at L2; the team's own loads
// and stores of it also go to L2, bypassing the compute unit's cache).
struct LdsCopy {
    lds_u32* h;
    __device__ __forceinline__ void zero(uint32_t b) { h[b] = 0u; }
    __device__ __forceinline__ void add(uint32_t k) {
        __hip_atomic_fetch_add(h + k, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __device__ __forceinline__ uint32_t get(uint32_t b) const { return h[b]; }
};
struct GlobalCopy {
    uint32_t* h;
    __device__ __forceinline__ void zero(uint32_t b) {
        __hip_atomic_store(h + b, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ void add(uint32_t k) {
        __hip_atomic_fetch_add(h + k, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ uint32_t get(uint32_t b) const {
        return __hip_atomic_load(h + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

// The team's bins are [b0, b0 + tb) of [0, bins).
struct BinRange {
    uint32_t bins, b0, tb;
};

template <class C>
__device__ __forceinline__ void count_key(C& c, int32_t k, const BinRange& r, bool& bad) {
    if ((uint32_t)k >= r.bins)
        bad = true;
    else if ((uint32_t)k - r.b0 < r.tb)
        c.add((uint32_t)k - r.b0);
}

// Zero the copy, count the keys of the team's balanced block that fall in
// its bins, add the non-zero bins into hist.  Returns whether a key was
// outside [0, bins).
template <int U, class C>
__device__ __forceinline__ bool team_histogram(C c, const int32_t* __restrict__ keys, int64_t n,
                                               const BinRange& bins, int64_t row, int64_t rows,
                                               int32_t* __restrict__ hist) {
    const int tid = threadIdx.x, P = blockDim.x;
    for (uint32_t b = tid; b < bins.tb; b += P) c.zero(b);
    __syncthreads();
    bool bad = false;
    const Range blk = bal_share(n, rows, row);
    if (blk.lo < blk.hi) {
        const int64_t a = blk.lo, e = blk.hi;
        const uintptr_t mis = reinterpret_cast<uintptr_t>(keys + a) & 15;
        int64_t head = (int64_t)(((16 - mis) & 15) / 4);
        if (head > e - a) head = e - a;
        if (tid < head) count_key(c, keys[a + tid], bins, bad);
        const int64_t p0 = a + head;
        const int64_t nv = (e - p0) / 4;
        using i32x4 = int32_t __attribute__((ext_vector_type(4)));
        const i32x4* __restrict__ vp = reinterpret_cast<const i32x4*>(keys + p0);
        int64_t v = tid;
        for (; v + (int64_t)(U - 1) * P < nv; v += (int64_t)U * P) {
            i32x4 r[U];
#pragma unroll
            for (int u = 0; u < U; ++u) r[u] = __builtin_nontemporal_load(vp + v + (int64_t)u * P);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) count_key(c, r[u][q], bins, bad);
        }
        for (; v < nv; v += P) {
            const i32x4 r = __builtin_nontemporal_load(vp + v);
#pragma unroll
            for (int q = 0; q < 4; ++q) count_key(c, r[q], bins, bad);
        }
        const int64_t t0 = p0 + nv * 4;
        if (tid < e - t0) count_key(c, keys[t0 + tid], bins, bad);
    }
    __syncthreads();
    for (uint32_t b = tid; b < bins.tb; b += P) {
        const uint32_t v = c.get(b);
        if (v)
            __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(hist) + bins.b0 + b, v,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return bad;
}

// Team k takes bin range k % tiles (tile_bins bins each, the last one
// shorter) and row block k / tiles of the keys.
template <int U>
__global__ __launch_bounds__(1024) void histogram_kernel(const int32_t* __restrict__ keys,
                                                         int64_t n, uint32_t bins,
                                                         uint32_t tiles, uint32_t tile_bins,
                                                         int32_t* __restrict__ hist, char* pool,
                                                         uint64_t pool_per_team,
                                                         uint32_t lds_cap, uint32_t* status) {
    extern __shared__ __align__(16) char arena[];
    __shared__ TeamStack st;
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    team_stack_init(&st, arena, lds_cap, pool ? pool + blockIdx.x * pool_per_team : nullptr,
                    pool_per_team);
    if (tid == 0) s_bad = 0;
    const uint32_t tile = blockIdx.x % tiles;
    BinRange r;
    r.bins = bins;
    r.b0 = tile * tile_bins;
    r.tb = r.b0 >= bins ? 0u : (bins - r.b0 < tile_bins ? bins - r.b0 : tile_bins);
    const int64_t rows = gridDim.x / tiles, row = blockIdx.x / tiles;
    void* h = team_alloc(&st, (uint64_t)r.tb * 4);
    if (!h) {   // the host sizes the pool so that this cannot happen
        if (tid == 0) __hip_atomic_fetch_or(status, 8u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const bool in_lds = static_cast<char*>(h) >= st.lds && static_cast<char*>(h) < st.lds + st.lds_cap;
    const bool bad = in_lds
                         ? team_histogram<U>(LdsCopy{(lds_u32*)h}, keys, n, r, row, rows, hist)
                         : team_histogram<U>(GlobalCopy{static_cast<uint32_t*>(h)}, keys, n, r,
                                             row, rows, hist);
    if (bad) s_bad = 1;
    __syncthreads();
    if (tid == 0 && s_bad) __hip_atomic_fetch_or(status, 4u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    team_free(&st, h, (uint64_t)r.tb * 4);
}

// Without a team copy: every key is an atomic add on hist itself (performed
// at the memory side's atomic units, coherent across the XCDs).  For bins
// far beyond LDS this is the cheaper reduction: no copy to zero and merge,
// and few keys meet on one bin.
template <int U>
__global__ __launch_bounds__(1024) void histogram_direct_kernel(const int32_t* __restrict__ keys,
                                                                int64_t n, uint32_t bins,
                                                                int32_t* __restrict__ hist,
                                                                uint32_t* status) {
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    const int64_t P = blockDim.x;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    uint32_t* h = reinterpret_cast<uint32_t*>(hist);
    bool bad = false;
    auto count = [&](int32_t k) {
        if ((uint32_t)k >= bins)
            bad = true;
        else
            __hip_atomic_fetch_add(h + k, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    const Range blk = bal_share(n, gridDim.x, blockIdx.x);
    if (blk.lo < blk.hi) {
        const int64_t a = blk.lo, e = blk.hi;
        const uintptr_t mis = reinterpret_cast<uintptr_t>(keys + a) & 15;
        int64_t head = (int64_t)(((16 - mis) & 15) / 4);
        if (head > e - a) head = e - a;
        if (tid < head) count(keys[a + tid]);
        const int64_t p0 = a + head;
        const int64_t nv = (e - p0) / 4;
        using i32x4 = int32_t __attribute__((ext_vector_type(4)));
        const i32x4* __restrict__ vp = reinterpret_cast<const i32x4*>(keys + p0);
        int64_t v = tid;
        for (; v + (U - 1) * P < nv; v += U * P) {
            i32x4 r[U];
#pragma unroll
            for (int u = 0; u < U; ++u) r[u] = __builtin_nontemporal_load(vp + v + u * P);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) count(r[u][q]);
        }
        for (; v < nv; v += P) {
            const i32x4 r = __builtin_nontemporal_load(vp + v);
#pragma unroll
            for (int q = 0; q < 4; ++q) count(r[q]);
        }
        const int64_t t0 = p0 + nv * 4;
        if (tid < e - t0) count(keys[t0 + tid]);
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (tid == 0 && s_bad) __hip_atomic_fetch_or(status, 4u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Global pool of the team copies that do not fit LDS: per (device, stream),
// grown on demand outside capture.
struct Pool {
    void* ptr = nullptr;
    uint64_t bytes = 0;
};
static std::mutex g_hmu;
static std::map<std::pair<int, hipStream_t>, Pool> g_pools;

static omprt_status pool_get(hipStream_t stream, uint64_t bytes, void** out) {
    int dev = 0;
    OMPRT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_hmu);
    Pool& p = g_pools[{dev, stream}];
    if (p.bytes < bytes) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        OMPRT_HIP(hipStreamIsCapturing(stream, &cs));
        if (cs != hipStreamCaptureStatusNone)
            return fail(OMPRT_ERR_INVALID, "stream is being captured and the histogram pool is "
                                           "too small: make the same call once before capturing");
        void* q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess)
            return fail(OMPRT_ERR_NOMEM, "histogram pool of %llu bytes", (unsigned long long)bytes);
        retire_device_memory(dev, p.ptr);   // a captured graph may still name it
        p.ptr = q;
        p.bytes = bytes;
    }
    *out = p.ptr;
    return OMPRT_OK;
}

void histogram_finalize() {
    std::lock_guard<std::mutex> lk(g_hmu);
    for (auto& kv : g_pools) {
        (void)hipSetDevice(kv.first.first);
        (void)hipFree(kv.second.ptr);
    }
    g_pools.clear();
}

// Dynamic LDS a team's copy may take: the device's LDS per workgroup (160 KiB
// on gfx950: 40 704 bins) less 1 KiB of room for the kernel's static LDS.
constexpr uint32_t kHistStaticLds = 1024;
static uint32_t hist_lds_cap() {
    static uint32_t cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024 - kHistStaticLds;
    if (!cached[dev]) {
        int bytes = 0;
        if (hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess ||
            bytes < 64 * 1024)
            bytes = 64 * 1024;
        cached[dev] = (uint32_t)bytes - kHistStaticLds;
    }
    return cached[dev];
}
// Bin ranges before atomics on hist: a key is read once per range, so ranges
// cost about 1.6 T keys/s / ranges at 2^28 keys (2: 808 G/s, 16: 125 G/s with
// 64 KiB ranges) against about 27 G keys/s for atomics on hist; 32 ranges
// keep a 2x margin.
constexpr uint32_t kMaxBinTiles = 32;

}  // namespace omprt

using namespace omprt;

extern "C" omprt_status omprt_histogram(const int32_t* d_keys, int64_t n, int32_t bins,
                                        int32_t* d_hist, const omprt_config* cfg,
                                        void* hip_stream) {
    if (n < 0 || n > ((int64_t)1 << 50))
        return fail(OMPRT_ERR_INVALID, "n = %lld outside 0..2^50", (long long)n);
    if (bins < 1 || bins > (1 << 28)) return fail(OMPRT_ERR_INVALID, "bins %d outside 1..2^28", bins);
    if (!d_hist) return fail(OMPRT_ERR_INVALID, "hist is NULL");
    if (n > 0 && !d_keys) return fail(OMPRT_ERR_INVALID, "keys is NULL with n > 0");
    if ((reinterpret_cast<uintptr_t>(d_keys) | reinterpret_cast<uintptr_t>(d_hist)) & 3)
        return fail(OMPRT_ERR_INVALID, "keys / hist not 4-byte aligned");
    int teams = 2 * device_cus(), threads = 512, unroll = 4;
    if (cfg) {
        if (cfg->num_teams < 0 || cfg->num_teams > 65535)
            return fail(OMPRT_ERR_INVALID, "num_teams %d", cfg->num_teams);
        if (cfg->threads_per_team &&
            (cfg->threads_per_team < 64 || cfg->threads_per_team > 1024 || cfg->threads_per_team % 64))
            return fail(OMPRT_ERR_INVALID, "threads_per_team %d", cfg->threads_per_team);
        if (cfg->unroll && cfg->unroll != 1 && cfg->unroll != 2 && cfg->unroll != 4)
            return fail(OMPRT_ERR_INVALID, "unroll %d (1, 2 or 4)", cfg->unroll);
        if (cfg->num_teams) teams = cfg->num_teams;
        if (cfg->threads_per_team) threads = cfg->threads_per_team;
        if (cfg->unroll) unroll = cfg->unroll;
    }
    const uint32_t flags = cfg ? cfg->flags : 0u;
    if ((flags & OMPRT_CFG_HIST_DIRECT) && (flags & OMPRT_CFG_HIST_TEAM_COPY))
        return fail(OMPRT_ERR_INVALID, "HIST_DIRECT and HIST_TEAM_COPY exclude each other");
    if (n == 0) return OMPRT_OK;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    // Bins that do not fit one team's LDS are cut into up to kMaxBinTiles
    // ranges, each counted by its own teams (every team reads its block of
    // the keys and counts those in its range: tiles x the key traffic, at
    // LDS atomic speed); past that, atomics on hist, or on request team
    // copies in the global pool (atomics at L2, then a merge).
    const uint32_t lds_bins = hist_lds_cap() / 4 / 4 * 4;
    uint32_t tiles = (uint32_t)((bins + lds_bins - 1) / lds_bins);
    uint32_t tile_bins = tiles > 1 ? (uint32_t)((bins + tiles - 1) / tiles + 3) / 4 * 4 : (uint32_t)bins;
    const bool direct = (flags & OMPRT_CFG_HIST_DIRECT) ||
                        (tiles > kMaxBinTiles && !(flags & OMPRT_CFG_HIST_TEAM_COPY));
    if (direct) {
        Workspace* ws = nullptr;
        if (omprt_status st = workspace_get(stream, 1, &ws)) return st;
        auto launch = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, dim3((unsigned)teams), dim3(threads), 0, stream, d_keys, n,
                               (uint32_t)bins, d_hist, ws->status());
        };
        switch (unroll) {
            case 1: launch(histogram_direct_kernel<1>); break;
            case 2: launch(histogram_direct_kernel<2>); break;
            default: launch(histogram_direct_kernel<4>); break;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "histogram launch: %s", hipGetErrorString(e));
        return OMPRT_OK;
    }
    const bool in_lds = tiles <= kMaxBinTiles;
    if (!in_lds) {
        tiles = 1;
        tile_bins = (uint32_t)bins;
    }
    const uint64_t hbytes = ((uint64_t)tile_bins * 4 + kSharedAlign - 1) / kSharedAlign * kSharedAlign;
    const int64_t rows = std::max<int64_t>(1, teams / (int64_t)tiles);
    const int64_t grid = rows * tiles;
    if (grid > INT32_MAX) return fail(OMPRT_ERR_INVALID, "grid too large");
    void* pool = nullptr;
    uint64_t per_team = 0;
    if (!in_lds) {
        per_team = (hbytes + 255) / 256 * 256;
        if (omprt_status st = pool_get(stream, per_team * (uint64_t)grid, &pool)) return st;
    }
    Workspace* ws = nullptr;
    if (omprt_status st = workspace_get(stream, 1, &ws)) return st;
    const uint32_t lds = in_lds ? (uint32_t)hbytes : 0u;
    hipError_t attr = hipSuccess;
    auto launch = [&](auto kernel) {
        if (lds > 64 * 1024)   // past the default dynamic LDS limit: ask for it
            attr = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (attr != hipSuccess) return;
        hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(threads), lds, stream, d_keys, n,
                           (uint32_t)bins, tiles, tile_bins, d_hist, static_cast<char*>(pool),
                           per_team, lds, ws->status());
    };
    switch (unroll) {
        case 1: launch(histogram_kernel<1>); break;
        case 2: launch(histogram_kernel<2>); break;
        default: launch(histogram_kernel<4>); break;
    }
    if (attr != hipSuccess)
        return fail(OMPRT_ERR_DEVICE, "histogram: %u bytes of LDS: %s", lds, hipGetErrorString(attr));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "histogram launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}
