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

// ---------------------------------------------------------------- partitioned bins
//
// Bins beyond one team's LDS copy, without reading the keys once per range:
// the keys are first partitioned by range (ranges of kPartBins bins, a
// power of two, so a key's range is key >> kPartLog2 and its place in the
// range key & (kPartBins - 1), kept as 16 bits), then each range's keys are
// counted in an LDS copy of that range alone.  Four kernels and a merge:
//   count    team t counts the valid keys of its balanced block per range
//            (LDS counters) -> cnt[r][t]
//   scan     one workgroup: off[r][t] = exclusive prefix of cnt in (r, t)
//            order, rstart[r] = off[r][0], rstart[R] = valid keys
//   scatter  team t re-reads its block and writes each valid key's 16-bit
//            place to part[off[r][t] + its rank among the team's keys of r]
//            (rank from an LDS cursor per range)
//   range    team (r, s) counts slice s of range r's part (S slices a range)
//            into an LDS copy of the range's bins; with S == 1 it adds the
//            copy into hist (it alone owns those bins), else it stores the
//            copy as partial s of those bins
//   merge    (S > 1) hist[b] += sum over s of partial[s][b]
// Key traffic: read twice, 16-bit places written once and read once (3 x
// the key bytes) against once per range for the range-by-range copies.
constexpr int kPartLog2 = 15;
constexpr uint32_t kPartBins = 1u << kPartLog2;   // 128 KiB of LDS counts
constexpr uint32_t kPartMaxRanges = 256;          // 8 388 608 bins
static_assert(kPartMaxRanges % 64 == 0 && kPartMaxRanges <= 1024, "one workgroup scans the ranges");
constexpr int kPartThreads = 512;

__device__ __forceinline__ void flag_bad(bool bad, int* s_bad, uint32_t* status) {
    if (bad) *s_bad = 1;
    __syncthreads();
    if (threadIdx.x == 0 && *s_bad)
        __hip_atomic_fetch_or(status, 4u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The valid keys of team t's balanced block of n, in order of position, to f
// (16-byte vectors, U in flight per lane); keys outside [0, bins) set bad.
template <int U, class F>
__device__ __forceinline__ void part_keys(const int32_t* __restrict__ keys, int64_t n,
                                          uint32_t bins, F&& f, bool& bad) {
    const int tid = threadIdx.x, P = blockDim.x;
    const Range blk = bal_share(n, gridDim.x, blockIdx.x);
    if (blk.lo >= blk.hi) return;
    auto one = [&](int32_t k) {
        if ((uint32_t)k >= bins)
            bad = true;
        else
            f((uint32_t)k);
    };
    const int64_t a = blk.lo, e = blk.hi;
    const uintptr_t mis = reinterpret_cast<uintptr_t>(keys + a) & 15;
    int64_t head = (int64_t)(((16 - mis) & 15) / 4);
    if (head > e - a) head = e - a;
    if (tid < head) one(keys[a + tid]);
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
            for (int q = 0; q < 4; ++q) one(r[u][q]);
    }
    for (; v < nv; v += P) {
        const i32x4 r = __builtin_nontemporal_load(vp + v);
#pragma unroll
        for (int q = 0; q < 4; ++q) one(r[q]);
    }
    const int64_t t0 = p0 + nv * 4;
    if (tid < e - t0) one(keys[t0 + tid]);
}

constexpr int kPartPerThread = 16;
constexpr int kPartTile = kPartThreads * kPartPerThread;

// LDS counters per range are kept in C copies, lane l adding to copy l % C:
// the lanes of a wave that meet on one range then meet on up to C addresses
// instead of one (same-address lanes of an LDS atomic are served one after
// another).  C = kPartCopies for up to 32 ranges, fewer above (R x C <= 256:
// the scatter scans R x C tile counts per tile, and with many ranges few
// lanes meet anyway).
constexpr uint32_t kPartCopies = 8;
__host__ __device__ constexpr uint32_t part_copies(uint32_t R) {
    return R <= 32 ? kPartCopies : R <= 64 ? 4u : R <= 128 ? 2u : 1u;
}

// Team t counts the valid keys of its balanced block per range.
__global__ __launch_bounds__(kPartThreads) void hist_part_count_kernel(
    const int32_t* __restrict__ keys, int64_t n, uint32_t bins, uint32_t R,
    uint32_t* __restrict__ cnt, uint32_t* status) {
    __shared__ uint32_t rc[kPartMaxRanges * kPartCopies];
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    const uint32_t C = part_copies(R);
    const uint32_t copy = (uint32_t)tid % C;
    if (tid == 0) s_bad = 0;
    for (uint32_t r = tid; r < R * C; r += blockDim.x) rc[r] = 0u;
    __syncthreads();
    bool bad = false;
    part_keys<4>(keys, n, bins,
                 [&](uint32_t k) {
                     __hip_atomic_fetch_add(rc + (k >> kPartLog2) * C + copy, 1u,
                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                 },
                 bad);
    __syncthreads();
    for (uint32_t r = tid; r < R; r += blockDim.x) {
        uint32_t c = 0;
        for (uint32_t q = 0; q < C; ++q) c += rc[r * C + q];
        cnt[(size_t)r * gridDim.x + blockIdx.x] = c;
    }
    flag_bad(bad, &s_bad, status);
}

// Inclusive scan of v over the workgroup (wave shuffles, then the wave totals
// in LDS); returns v's inclusive prefix, *total the workgroup's sum.  Every
// thread of the workgroup calls it; the workgroup is whole waves.
__device__ inline int64_t block_scan_inclusive(int64_t v, int64_t* wsum, int64_t* total) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    int64_t inc = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t o = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += o;
    }
    if (lane == kWave - 1) wsum[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        int64_t w = lane < nw ? wsum[lane] : 0;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int64_t o = __shfl_up(w, d, kWave);
            if (lane >= d) w += o;
        }
        if (lane < nw) wsum[lane] = w;   // inclusive totals of waves 0..lane
    }
    __syncthreads();
    const int64_t r = inc + (wave > 0 ? wsum[wave - 1] : 0);
    *total = wsum[nw - 1];
    __syncthreads();   // wsum is reused by the next call
    return r;
}

// Places within each range: workgroup r scans range r's T team counts
// (cnt[r T + t], coalesced, a workgroup-wide piece at a time) into
// off[r T + t] = the keys teams 0..t-1 put in range r, and leaves the
// range's total in rstart[r].
__global__ __launch_bounds__(1024) void hist_part_scan_range_kernel(const uint32_t* __restrict__ cnt,
                                                                    uint32_t T,
                                                                    int64_t* __restrict__ off,
                                                                    int64_t* __restrict__ rstart) {
    __shared__ int64_t wsum[kMaxWaves];
    const size_t r = blockIdx.x;
    int64_t carry = 0;
    for (uint32_t t0 = 0; t0 < T; t0 += blockDim.x) {
        const uint32_t t = t0 + threadIdx.x;
        const int64_t v = t < T ? cnt[r * T + t] : 0;
        int64_t tot = 0;
        const int64_t inc = block_scan_inclusive(v, wsum, &tot);
        if (t < T) off[r * T + t] = carry + inc - v;
        carry += tot;
    }
    if (threadIdx.x == 0) rstart[r] = carry;
}

// Range starts: rstart[0..R) holds the range totals on entry and their
// exclusive prefix sums on return, rstart[R] the number of valid keys.  One
// workgroup; every total is read before any is written.
__global__ __launch_bounds__(1024) void hist_part_scan_start_kernel(uint32_t R,
                                                                    int64_t* __restrict__ rstart) {
    __shared__ int64_t wsum[kMaxWaves];
    const uint32_t r = threadIdx.x;   // R <= blockDim.x
    const int64_t v = r < R ? rstart[r] : 0;
    int64_t tot = 0;
    const int64_t inc = block_scan_inclusive(v, wsum, &tot);
    if (r < R) rstart[r] = inc - v;
    if (r == 0) rstart[R] = tot;
}

// Scatter, a tile of kPartTile keys at a time: the tile's valid keys are
// ranked within their range (LDS counters), the ranges' tile
// counts scanned, and the 16-bit places sorted by range into an LDS buffer;
// then consecutive lanes store consecutive places of one range to
// consecutive positions of its bucket, so the stores come as contiguous runs
// (not one 2-byte store per key anywhere in memory).  Within its part of a
// range's bucket a team writes its keys tile by tile; the count kernel
// fixed how many there are.
__global__ __launch_bounds__(kPartThreads) void hist_part_scatter_kernel(
    const int32_t* __restrict__ keys, int64_t n, uint32_t bins, uint32_t R,
    const int64_t* __restrict__ off, const int64_t* __restrict__ rstart,
    uint16_t* __restrict__ part) {
    const uint32_t C = part_copies(R);
    __shared__ int64_t base[kPartMaxRanges];
    __shared__ uint32_t tcnt[kPartMaxRanges * kPartCopies];       // [range][copy]
    __shared__ uint32_t toff[kPartMaxRanges * kPartCopies + 1];   // exclusive scan of tcnt
    __shared__ uint16_t buf_place[kPartTile];
    __shared__ uint16_t buf_range[kPartTile];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), P = blockDim.x;
    const uint32_t copy = (uint32_t)tid % C;
    const uint32_t RC = R * C;
    for (uint32_t r = tid; r < R; r += P)
        base[r] = rstart[r] + off[(size_t)r * gridDim.x + blockIdx.x];
    const Range blk = bal_share(n, gridDim.x, blockIdx.x);
    // the next tile's keys are loaded while this one is sorted and stored
    uint32_t kn[kPartPerThread];
    auto load_tile = [&](int64_t t0) {
#pragma unroll
        for (int q = 0; q < kPartPerThread; ++q) {
            const int64_t i = t0 + (int64_t)q * P + tid;
            kn[q] = i < blk.hi ? (uint32_t)__builtin_nontemporal_load(keys + i) : 0xFFFFFFFFu;
        }
    };
    if (blk.lo < blk.hi) load_tile(blk.lo);
    for (int64_t t0 = blk.lo; t0 < blk.hi; t0 += kPartTile) {
        for (uint32_t e = tid; e < RC; e += P) tcnt[e] = 0u;
        uint32_t kr[kPartPerThread], rank[kPartPerThread];
#pragma unroll
        for (int q = 0; q < kPartPerThread; ++q) kr[q] = kn[q];
        if (t0 + kPartTile < blk.hi) load_tile(t0 + kPartTile);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPartPerThread; ++q)
            if (kr[q] < bins)
                rank[q] = __hip_atomic_fetch_add(tcnt + (kr[q] >> kPartLog2) * C + copy, 1u,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __syncthreads();
        if (tid < kWave) {   // exclusive scan of the tile counts in (range, copy) order, one wave
            uint32_t carry = 0;
            for (uint32_t c0 = 0; c0 < RC; c0 += kWave) {
                const uint32_t e = c0 + lane;
                const uint32_t v = e < RC ? tcnt[e] : 0u;
                uint32_t inc = v;
#pragma unroll
                for (int d = 1; d < kWave; d <<= 1) {
                    const uint32_t o = __shfl_up(inc, d, kWave);
                    if (lane >= d) inc += o;
                }
                if (e < RC) toff[e] = carry + inc - v;
                carry += __shfl(inc, kWave - 1, kWave);
            }
            if (lane == 0) toff[RC] = carry;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPartPerThread; ++q)
            if (kr[q] < bins) {
                const uint32_t r = kr[q] >> kPartLog2;
                const uint32_t at = toff[r * C + copy] + rank[q];
                buf_place[at] = (uint16_t)(kr[q] & (kPartBins - 1));
                buf_range[at] = (uint16_t)r;
            }
        __syncthreads();
        // a range's keys of the tile are buf[toff[r C] .. toff[(r + 1) C])
        const uint32_t total = toff[RC];
        for (uint32_t at = tid; at < total; at += P) {
            const uint32_t r = buf_range[at];
            part[base[r] + (at - toff[r * C])] = buf_place[at];
        }
        __syncthreads();
        for (uint32_t r = tid; r < R; r += P) base[r] += toff[(r + 1) * C] - toff[r * C];
        __syncthreads();
    }
}

// Team (r, s): slice s of S of range r's places.  out is hist (S == 1) or
// the partials, S x bins.
__global__ __launch_bounds__(kPartThreads) void hist_part_range_kernel(
    const uint16_t* __restrict__ part, const int64_t* __restrict__ rstart, uint32_t bins,
    uint32_t S, uint32_t* __restrict__ out) {
    extern __shared__ __align__(16) char arena[];
    lds_u32* h = (lds_u32*)arena;
    const int tid = threadIdx.x, P = blockDim.x;
    const uint32_t r = blockIdx.x / S, s = blockIdx.x % S;
    const uint32_t b0 = r << kPartLog2;
    const uint32_t tb = bins - b0 < kPartBins ? bins - b0 : kPartBins;
    for (uint32_t b = tid; b < tb; b += P) h[b] = 0u;
    __syncthreads();
    const Range sl = bal_share(rstart[r + 1] - rstart[r], S, s);
    const int64_t a = rstart[r] + sl.lo, e = rstart[r] + sl.hi;
    auto add = [&](uint32_t j) {
        __hip_atomic_fetch_add(h + j, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    if (a < e) {
        const uintptr_t mis = reinterpret_cast<uintptr_t>(part + a) & 15;
        int64_t head = (int64_t)(((16 - mis) & 15) / 2);
        if (head > e - a) head = e - a;
        if (tid < head) add(part[a + tid]);
        const int64_t p0 = a + head;
        const int64_t nv = (e - p0) / 8;
        using u32x4v = uint32_t __attribute__((ext_vector_type(4)));
        const u32x4v* __restrict__ vp = reinterpret_cast<const u32x4v*>(part + p0);
        constexpr int U = 4;
        int64_t v = tid;
        for (; v + (int64_t)(U - 1) * P < nv; v += (int64_t)U * P) {
            u32x4v w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) w[u] = __builtin_nontemporal_load(vp + v + (int64_t)u * P);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    add(w[u][q] & 0xFFFFu);
                    add(w[u][q] >> 16);
                }
        }
        for (; v < nv; v += P) {
            const u32x4v w = __builtin_nontemporal_load(vp + v);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                add(w[q] & 0xFFFFu);
                add(w[q] >> 16);
            }
        }
        const int64_t t0 = p0 + nv * 8;
        if (tid < e - t0) add(part[t0 + tid]);
    }
    __syncthreads();
    if (S == 1) {
        for (uint32_t b = tid; b < tb; b += P) {
            const uint32_t c = h[b];
            if (c) out[b0 + b] += c;
        }
    } else {
        uint32_t* o = out + (size_t)s * bins + b0;
        for (uint32_t b = tid; b < tb; b += P) o[b] = h[b];
    }
}

__global__ void hist_part_merge_kernel(const uint32_t* __restrict__ partial, uint32_t S,
                                       uint32_t bins, uint32_t* __restrict__ hist) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bins) return;
    uint32_t c = 0;
    for (uint32_t s = 0; s < S; ++s) c += partial[(size_t)s * bins + b];
    if (c) hist[b] += c;
}

// Tile-sorted partition, up to kTsortMaxRanges ranges: every tile of
// kPartTile keys of a team's balanced block is ranked and sorted by range in
// LDS as in the scatter above, but stored whole into a slot of its own,
// kTsortSlot places: range r's run starts on a 16-byte boundary (each run is
// padded with kTsortPad to a multiple of eight places) and the runs' starts,
// in 16-byte vectors, go to tstart[g (R + 1) + r] (g = team x tiles per
// team + tile; entry R is the slot's end).  No count pass and no scan
// across teams: the range kernel then reads range r's run of every tile.
// Key traffic: read once, places written once and read once (2 x the key
// bytes), against three times for the partition above; the runs of a tile
// are 8192 / R places long on average (64 at 128 ranges), and the padding
// adds at most 8 R places a tile (12.5 % at 128 ranges).
constexpr uint32_t kTsortMaxRanges = 128;
constexpr uint32_t kTsortSlot = kPartTile + 8 * kTsortMaxRanges;   // places, 16-byte multiple
constexpr uint32_t kTsortPad = 0xFFFFu;                            // never a place (< kPartBins)
static_assert(kTsortSlot % 8 == 0 && kTsortSlot / 8 < 65536, "slot of whole 16-byte vectors");

__global__ __launch_bounds__(kPartThreads) void hist_tsort_scatter_kernel(
    const int32_t* __restrict__ keys, int64_t n, uint32_t bins, uint32_t R, uint32_t NT,
    uint16_t* __restrict__ part, uint16_t* __restrict__ tstart, uint32_t* status) {
    const uint32_t C = part_copies(R);
    __shared__ uint32_t tcnt[kTsortMaxRanges * kPartCopies];       // [range][copy]
    __shared__ uint32_t toff[kTsortMaxRanges * kPartCopies + 1];   // exclusive scan of tcnt
    __shared__ uint32_t pst[kTsortMaxRanges + 1];                  // padded run starts
    __shared__ uint32_t wtot[kTsortMaxRanges * kPartCopies / kWave];
    __shared__ __align__(16) uint16_t buf[kTsortSlot];
    __shared__ int s_bad;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), P = blockDim.x;
    const uint32_t copy = (uint32_t)tid % C;
    const uint32_t RC = R * C;
    if (tid == 0) s_bad = 0;
    bool bad = false;
    const Range blk = bal_share(n, gridDim.x, blockIdx.x);
    // the next tile's keys are loaded while this one is sorted and stored
    // (nothing reads them before then); positions past the block read as
    // 0xFFFFFFFF (not a valid key)
    uint32_t kn[kPartPerThread];
    auto load_tile = [&](int64_t t0) {
#pragma unroll
        for (int q = 0; q < kPartPerThread; ++q) {
            const int64_t i = t0 + (int64_t)q * P + tid;
            kn[q] = i < blk.hi ? (uint32_t)__builtin_nontemporal_load(keys + i) : 0xFFFFFFFFu;
        }
    };
    if (blk.lo < blk.hi) load_tile(blk.lo);
    uint32_t j = 0;
    for (int64_t t0 = blk.lo; t0 < blk.hi; t0 += kPartTile, ++j) {
        for (uint32_t e = tid; e < RC; e += P) tcnt[e] = 0u;
        uint32_t kr[kPartPerThread], rank[kPartPerThread];
#pragma unroll
        for (int q = 0; q < kPartPerThread; ++q) kr[q] = kn[q];
        if (t0 + kPartTile < blk.hi) load_tile(t0 + kPartTile);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPartPerThread; ++q) {
            if (kr[q] < bins)
                rank[q] = __hip_atomic_fetch_add(tcnt + (kr[q] >> kPartLog2) * C + copy, 1u,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else if (t0 + (int64_t)q * P + tid < blk.hi)
                bad = true;
        }
        __syncthreads();
        // exclusive scan of the tile counts in (range, copy) order: entry e
        // by thread e, the waves' totals through LDS
        uint32_t v = 0, inc = 0;
        if ((uint32_t)tid < RC) {
            v = tcnt[tid];
            inc = v;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t o = __shfl_up(inc, d, kWave);
                if (lane >= d) inc += o;
            }
            if (lane == kWave - 1 || (uint32_t)tid == RC - 1) wtot[tid / kWave] = inc;
        }
        __syncthreads();
        if ((uint32_t)tid < RC) {
            uint32_t before = 0;
            for (int w = 0; w < tid / kWave; ++w) before += wtot[w];
            toff[tid] = before + inc - v;
            if ((uint32_t)tid == RC - 1) toff[RC] = before + inc;
        }
        __syncthreads();
        if (tid < kWave) {   // padded run starts: each run rounded up to eight places
            uint32_t carry = 0;
            for (uint32_t r0 = 0; r0 <= R; r0 += kWave) {
                const uint32_t r = r0 + (uint32_t)lane;
                const uint32_t len = r < R ? toff[(r + 1) * C] - toff[r * C] : 0u;
                const uint32_t pl = (len + 7u) & ~7u;
                uint32_t inc = pl;
#pragma unroll
                for (int d = 1; d < kWave; d <<= 1) {
                    const uint32_t o = __shfl_up(inc, d, kWave);
                    if (lane >= d) inc += o;
                }
                if (r <= R) pst[r] = carry + inc - pl;   // entry R: the padded total
                carry += __shfl(inc, kWave - 1, kWave);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPartPerThread; ++q)
            if (kr[q] < bins) {
                const uint32_t r = kr[q] >> kPartLog2;
                buf[pst[r] + toff[r * C + copy] - toff[r * C] + rank[q]] =
                    (uint16_t)(kr[q] & (kPartBins - 1));
            }
        for (uint32_t e = (uint32_t)tid; e < R * 8; e += P) {   // the padding after each run
            const uint32_t r = e / 8, u = e % 8;
            const uint32_t at = pst[r] + (toff[(r + 1) * C] - toff[r * C]) + u;
            if (at < pst[r + 1]) buf[at] = (uint16_t)kTsortPad;
        }
        __syncthreads();
        const size_t g = (size_t)blockIdx.x * NT + j;
        u32x4* __restrict__ slot = reinterpret_cast<u32x4*>(part + g * kTsortSlot);
        const u32x4* lb = reinterpret_cast<const u32x4*>(buf);
        for (uint32_t v = tid; v < pst[R] / 8; v += P) slot[v] = lb[v];
        if ((uint32_t)tid <= R) tstart[g * (R + 1) + tid] = (uint16_t)(pst[tid] / 8);
        // the next tile rewrites pst and buf only after two more barriers
    }
    for (uint32_t e = (uint32_t)tid; e < (NT - j) * (R + 1); e += P)   // empty tiles
        tstart[((size_t)blockIdx.x * NT + j) * (R + 1) + e] = 0;
    flag_bad(bad, &s_bad, status);
}

// Team (r, s): range r's runs in slice s of the G tile slots, each group of
// SW lanes (a wave, or half of one when runs are short) sixteen tiles at a
// time, one 16-byte vector of each in flight per lane (the LDS copy of the
// range allows one team a CU, so registers are plentiful).  out is hist (S ==
// 1) or the partials, S x bins.
template <int SW>
__global__ __launch_bounds__(kPartThreads) void hist_tsort_range_kernel(
    const uint16_t* __restrict__ part, const uint16_t* __restrict__ tstart, int64_t G,
    uint32_t R, uint32_t bins, uint32_t S, uint32_t* __restrict__ out) {
    extern __shared__ __align__(16) char arena[];
    lds_u32* h = (lds_u32*)arena;
    const int tid = threadIdx.x, lane = tid & (SW - 1), P = blockDim.x;
    const int64_t W = P / SW, wave = tid / SW;
    const uint32_t r = blockIdx.x / S, s = blockIdx.x % S;
    const uint32_t b0 = r << kPartLog2;
    const uint32_t tb = bins - b0 < kPartBins ? bins - b0 : kPartBins;
    for (uint32_t b = tid; b < tb; b += P) h[b] = 0u;
    __syncthreads();
    auto add = [&](uint32_t j) {
        if (j != kTsortPad)
            __hip_atomic_fetch_add(h + j, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    const Range sl = bal_share(G, S, s);
    constexpr int K = SW < 16 ? SW : 16;   // tiles of a group: one lane fetches each
    const int64_t step = K * W;
    // run starts and lengths of a group of K tiles (g0, g0 + W, ...): the next
    // group's are loaded while this group's places stream in
    // (lane k of the group loads tile k's entries; the group shares them)
    static_assert(K <= SW, "a lane per tile of the group");
    const int first = (tid & (kWave - 1)) - lane;   // the group's first lane in the wave
    uint32_t st[K], nv[K];
    auto fetch = [&](int64_t g0) {
        const int64_t g = g0 + (int64_t)lane * W;
        uint32_t a = 0, b = 0;
        if (lane < K && g < sl.hi) {
            a = tstart[g * (R + 1) + r];
            b = tstart[g * (R + 1) + r + 1];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            st[k] = (uint32_t)__shfl((int)a, first + k, kWave);
            nv[k] = (uint32_t)__shfl((int)b, first + k, kWave) - st[k];
        }
    };
    int64_t g0 = sl.lo + wave;
    if (g0 < sl.hi) fetch(g0);
    for (; g0 < sl.hi; g0 += step) {
        uint32_t cst[K], cnv[K], mx = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            cst[k] = st[k];
            cnv[k] = nv[k];
            mx = cnv[k] > mx ? cnv[k] : mx;
        }
        if (g0 + step < sl.hi) fetch(g0 + step);
        for (uint32_t i = lane; i < mx; i += SW) {
            u32x4 w[K];
#pragma unroll
            for (int k = 0; k < K; ++k)
                w[k] = i < cnv[k] ? __builtin_nontemporal_load(
                                        reinterpret_cast<const u32x4*>(part + (g0 + k * W) * kTsortSlot) +
                                        cst[k] + i)
                                  : u32x4{~0u, ~0u, ~0u, ~0u};
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    add(w[k][q] & 0xFFFFu);
                    add(w[k][q] >> 16);
                }
        }
    }
    __syncthreads();
    if (S == 1) {
        for (uint32_t b = tid; b < tb; b += P) {
            const uint32_t c = h[b];
            if (c) out[b0 + b] += c;
        }
    } else {
        uint32_t* o = out + (size_t)s * bins + b0;
        for (uint32_t b = tid; b < tb; b += P) o[b] = h[b];
    }
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
// Ranges the default takes before partitioning the keys: ranges cost one
// read of the keys each, the partition about three plus its passes' fixed
// costs; at 2^28 uniform keys 3 ranges ran at 441 G keys/s against 267 for
// the partition, 7 ranges at 197 against 319.
constexpr uint32_t kDefaultMaxBinTiles = 4;
// LDS ranges the default takes before the tile sort (which reads the keys
// once and moves 2-byte places twice): at 2^28 uniform keys 3 ranges ran at
// 444 G keys/s against 535 for the tile sort, 2 ranges at 793 against 432.
constexpr uint32_t kDefaultMaxTsortTiles = 2;

// Partitioned bins (count, scan, scatter, range, merge), teams x 512
// threads for the passes over the keys.
static omprt_status histogram_partitioned(const int32_t* d_keys, int64_t n, uint32_t bins,
                                          int32_t* d_hist, int teams, hipStream_t stream) {
    const uint32_t R = (bins + kPartBins - 1) >> kPartLog2;
    if (R > kPartMaxRanges)
        return fail(OMPRT_ERR_INVALID, "partitioned histogram: %u bins above %u", bins,
                    kPartMaxRanges * kPartBins);
    const uint32_t T = (uint32_t)teams;
    uint32_t S = (uint32_t)((2 * device_cus() + R - 1) / R);
    S = std::min<uint32_t>(std::max<uint32_t>(S, 1u), 64u);
    auto up = [](uint64_t b) { return (b + 255) / 256 * 256; };
    const uint64_t b_part = up((uint64_t)n * 2), b_cnt = up((uint64_t)R * T * 4),
                   b_off = up((uint64_t)R * T * 8), b_rs = up((uint64_t)(R + 1) * 8),
                   b_partial = S > 1 ? up((uint64_t)S * bins * 4) : 0;
    void* pool = nullptr;
    if (omprt_status st = pool_get(stream, b_part + b_cnt + b_off + b_rs + b_partial, &pool))
        return st;
    char* p = static_cast<char*>(pool);
    uint16_t* part = reinterpret_cast<uint16_t*>(p);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(p + b_part);
    int64_t* off = reinterpret_cast<int64_t*>(p + b_part + b_cnt);
    int64_t* rstart = reinterpret_cast<int64_t*>(p + b_part + b_cnt + b_off);
    uint32_t* partial = reinterpret_cast<uint32_t*>(p + b_part + b_cnt + b_off + b_rs);
    Workspace* ws = nullptr;
    if (omprt_status st = workspace_get(stream, 1, &ws)) return st;
    uint32_t* hist = reinterpret_cast<uint32_t*>(d_hist);
    hipLaunchKernelGGL(hist_part_count_kernel, dim3(T), dim3(kPartThreads), 0, stream, d_keys, n,
                       bins, R, cnt, ws->status());
    const uint32_t scan_threads = std::min<uint32_t>((T + kWave - 1) / kWave * kWave, 1024u);
    hipLaunchKernelGGL(hist_part_scan_range_kernel, dim3(R), dim3(scan_threads), 0, stream, cnt,
                       T, off, rstart);
    hipLaunchKernelGGL(hist_part_scan_start_kernel, dim3(1), dim3(kPartMaxRanges), 0, stream, R,
                       rstart);
    hipLaunchKernelGGL(hist_part_scatter_kernel, dim3(T), dim3(kPartThreads), 0, stream, d_keys,
                       n, bins, R, off, rstart, part);
    const uint32_t lds = std::min(bins, kPartBins) * 4;
    if (lds > 64 * 1024) {   // past the default dynamic LDS limit: ask for it
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(hist_part_range_kernel),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return fail(OMPRT_ERR_DEVICE, "histogram: %u bytes of LDS: %s", lds,
                        hipGetErrorString(e));
    }
    hipLaunchKernelGGL(hist_part_range_kernel, dim3(R * S), dim3(kPartThreads), lds, stream, part,
                       rstart, bins, S, S > 1 ? partial : hist);
    if (S > 1)
        hipLaunchKernelGGL(hist_part_merge_kernel, dim3((bins + 255) / 256), dim3(256), 0, stream,
                           partial, S, bins, hist);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "histogram launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}

// Tile-sorted bins (scatter into tile slots, range, merge), up to
// kTsortMaxRanges ranges; teams x 512 threads for the pass over the keys.
static omprt_status histogram_tsorted(const int32_t* d_keys, int64_t n, uint32_t bins,
                                      int32_t* d_hist, int teams, hipStream_t stream) {
    const uint32_t R = (bins + kPartBins - 1) >> kPartLog2;
    if (R > kTsortMaxRanges)
        return fail(OMPRT_ERR_INVALID, "tile-sorted histogram: %u bins above %u", bins,
                    kTsortMaxRanges * kPartBins);
    // no more teams than tiles: a team without keys would still own a slot
    const uint32_t T = (uint32_t)std::min<int64_t>(teams, (n + kPartTile - 1) / kPartTile);
    const int64_t per_team = (n + T - 1) / T;
    const uint32_t NT = (uint32_t)std::max<int64_t>(1, (per_team + kPartTile - 1) / kPartTile);
    const int64_t G = (int64_t)T * NT;
    uint32_t S = (uint32_t)((2 * device_cus() + R - 1) / R);
    S = std::min<uint32_t>(std::max<uint32_t>(S, 1u), 64u);
    auto up = [](uint64_t b) { return (b + 255) / 256 * 256; };
    const uint64_t b_part = up((uint64_t)G * kTsortSlot * 2),
                   b_ts = up((uint64_t)G * (R + 1) * 2),
                   b_partial = S > 1 ? up((uint64_t)S * bins * 4) : 0;
    void* pool = nullptr;
    if (omprt_status st = pool_get(stream, b_part + b_ts + b_partial, &pool)) return st;
    char* p = static_cast<char*>(pool);
    uint16_t* part = reinterpret_cast<uint16_t*>(p);
    uint16_t* tstart = reinterpret_cast<uint16_t*>(p + b_part);
    uint32_t* partial = reinterpret_cast<uint32_t*>(p + b_part + b_ts);
    Workspace* ws = nullptr;
    if (omprt_status st = workspace_get(stream, 1, &ws)) return st;
    uint32_t* hist = reinterpret_cast<uint32_t*>(d_hist);
    hipLaunchKernelGGL(hist_tsort_scatter_kernel, dim3(T), dim3(kPartThreads), 0, stream, d_keys,
                       n, bins, R, NT, part, tstart, ws->status());
    // runs average kPartTile / R places: from 16 ranges on (64 vectors or
    // fewer) half a wave takes a tile, from 48 on a quarter, from 96 an eighth
    const void* range_kernel =
        R >= 96   ? reinterpret_cast<const void*>(hist_tsort_range_kernel<8>)
        : R >= 48 ? reinterpret_cast<const void*>(hist_tsort_range_kernel<16>)
        : R >= 16 ? reinterpret_cast<const void*>(hist_tsort_range_kernel<32>)
                  : reinterpret_cast<const void*>(hist_tsort_range_kernel<64>);
    const uint32_t lds = std::min(bins, kPartBins) * 4;
    if (lds > 64 * 1024) {   // past the default dynamic LDS limit: ask for it
        const hipError_t e =
            hipFuncSetAttribute(range_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return fail(OMPRT_ERR_DEVICE, "histogram: %u bytes of LDS: %s", lds,
                        hipGetErrorString(e));
    }
    uint32_t* dst = S > 1 ? partial : hist;
    if (R >= 96)
        hipLaunchKernelGGL(hist_tsort_range_kernel<8>, dim3(R * S), dim3(kPartThreads), lds,
                           stream, part, tstart, G, R, bins, S, dst);
    else if (R >= 48)
        hipLaunchKernelGGL(hist_tsort_range_kernel<16>, dim3(R * S), dim3(kPartThreads), lds,
                           stream, part, tstart, G, R, bins, S, dst);
    else if (R >= 16)
        hipLaunchKernelGGL(hist_tsort_range_kernel<32>, dim3(R * S), dim3(kPartThreads), lds,
                           stream, part, tstart, G, R, bins, S, dst);
    else
        hipLaunchKernelGGL(hist_tsort_range_kernel<64>, dim3(R * S), dim3(kPartThreads), lds,
                           stream, part, tstart, G, R, bins, S, dst);
    if (S > 1)
        hipLaunchKernelGGL(hist_part_merge_kernel, dim3((bins + 255) / 256), dim3(256), 0, stream,
                           partial, S, bins, hist);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "histogram launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}

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
    const uint32_t forced = flags & (OMPRT_CFG_HIST_DIRECT | OMPRT_CFG_HIST_TEAM_COPY |
                                     OMPRT_CFG_HIST_PARTITION | OMPRT_CFG_HIST_RANGES |
                                     OMPRT_CFG_HIST_TILE_SORT);
    if (forced & (forced - 1))
        return fail(OMPRT_ERR_INVALID, "at most one of HIST_DIRECT, HIST_TEAM_COPY, "
                                       "HIST_PARTITION, HIST_RANGES, HIST_TILE_SORT");
    if ((flags & OMPRT_CFG_HIST_PARTITION) && bins > (int64_t)kPartMaxRanges * kPartBins)
        return fail(OMPRT_ERR_INVALID, "HIST_PARTITION takes up to %u bins",
                    kPartMaxRanges * kPartBins);
    if ((flags & OMPRT_CFG_HIST_TILE_SORT) && bins > (int64_t)kTsortMaxRanges * kPartBins)
        return fail(OMPRT_ERR_INVALID, "HIST_TILE_SORT takes up to %u bins",
                    kTsortMaxRanges * kPartBins);
    if (n == 0) return OMPRT_OK;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    // Bins that do not fit one team's LDS: up to four ranges of bins, each
    // counted by its own teams (every team reads its block of the keys and
    // counts those in its range); from five ranges on, the keys partitioned by
    // range first: up to kTsortMaxRanges ranges each tile sorted by range into
    // a slot of its own (keys read once, 16-bit places written and read
    // once), then up to kPartMaxRanges x kPartBins bins partitioned across
    // teams (keys read twice), both within 16 GiB of places; past that,
    // atomics on hist.  On request: ranges up to kMaxBinTiles of them, team
    // copies in the global pool (atomics at L2, then a merge), either
    // partition, or atomics on hist for any bin count.
    const uint32_t lds_bins = hist_lds_cap() / 4 / 4 * 4;
    uint32_t tiles = (uint32_t)((bins + lds_bins - 1) / lds_bins);
    uint32_t tile_bins = tiles > 1 ? (uint32_t)((bins + tiles - 1) / tiles + 3) / 4 * 4 : (uint32_t)bins;
    const bool part_fits = bins <= (int64_t)kPartMaxRanges * kPartBins &&
                           (uint64_t)n * 2 <= ((uint64_t)16 << 30);
    const bool tsort_fits = part_fits && bins <= (int64_t)kTsortMaxRanges * kPartBins;
    if ((flags & OMPRT_CFG_HIST_TILE_SORT) ||
        (!forced && tiles > kDefaultMaxTsortTiles && tsort_fits))
        return histogram_tsorted(d_keys, n, (uint32_t)bins, d_hist, teams, stream);
    if ((flags & OMPRT_CFG_HIST_PARTITION) ||
        (!forced && tiles > kDefaultMaxBinTiles && part_fits))
        return histogram_partitioned(d_keys, n, (uint32_t)bins, d_hist, teams, stream);
    const bool direct = (flags & OMPRT_CFG_HIST_DIRECT) ||
                        (tiles > kMaxBinTiles && !(flags & OMPRT_CFG_HIST_TEAM_COPY)) ||
                        (!forced && tiles > kDefaultMaxBinTiles);
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
