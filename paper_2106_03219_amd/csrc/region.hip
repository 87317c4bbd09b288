// region.hip -- a parallel region with two worksharing loops, the first
// with or without its implicit barrier (nowait):
//   loop 1, schedule(static, c1) [nowait]:     y[i] = fmaf(a, x[i], y[i])
//   loop 2, schedule(static, c2), reduction(+: s):  s += y[i]
// Both loops take the same distribute schedule, so team k executes the same
// iterations in both and no team waits for another between them.  Inside a
// team, loop 2 reads y that loop 1 wrote: with the barrier any thread may
// read any element; without it only the thread that wrote an element may
// read it, which OpenMP guarantees when the two loops have the same static
// schedule (same iteration count and chunk): every iteration goes to the
// same thread in both, and each thread's own stores precede its loads.
// With c1 != c2 the entry point therefore refuses nowait.
#include <algorithm>

#include "axpy.h"
#include "device.h"
#include "launch.h"
#include "runtime.h"
#include "sched.h"

namespace omprt {

// One chunk [lo, hi) of the calling thread, read only: elements up to
// 16-byte alignment, then 16-byte vectors eight in flight, then the tail.
__device__ __forceinline__ void sum_range(const float* __restrict__ y, int64_t lo, int64_t hi,
                                          ff_t& acc) {
    const uintptr_t mis = reinterpret_cast<uintptr_t>(y + lo) & 15;
    int64_t head = (int64_t)(((16 - mis) & 15) / 4);
    if (head > hi - lo) head = hi - lo;
    int64_t i = lo;
    for (; i < lo + head; ++i) comp_add(acc, y[i]);
    const float4* __restrict__ yv = reinterpret_cast<const float4*>(y + i);
    const int64_t nv = (hi - i) / 4;
    int64_t j = 0;
    for (; j + 8 <= nv; j += 8) {
        float4 r[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) r[u] = yv[j + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            comp_add(acc, r[u].x);
            comp_add(acc, r[u].y);
            comp_add(acc, r[u].z);
            comp_add(acc, r[u].w);
        }
    }
    for (; j < nv; ++j) {
        const float4 r = yv[j];
        comp_add(acc, r.x);
        comp_add(acc, r.y);
        comp_add(acc, r.z);
        comp_add(acc, r.w);
    }
    for (i += nv * 4; i < hi; ++i) comp_add(acc, y[i]);
}

// Loop 2's share of a union (axpy_run_union's geometry: under nowait the lane
// that loads a block of y is the lane that stored it in loop 1), else the
// lane alone.
__device__ __forceinline__ void sum_run_union(const float* __restrict__ y, int64_t lo, int64_t hi,
                                              f32x4* __restrict__ xs, f32x4* __restrict__ ys,
                                              ff_t& acc) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t next_lo = __shfl_down(lo, 1, kWave);
    const bool joined = lane == kWave - 1 || hi == next_lo;
    if (__ballot(joined) != ~0ull) {
        sum_range(y, lo, hi, acc);
        return;
    }
    axpy_union_lines<false>(0.0f, nullptr, const_cast<float*>(y), lo, hi, xs, ys, &acc);
}

// Chunk size 1: thread t reads lo + t, lo + t + P, ... (coalesced across
// the wave), eight rows in flight.
__device__ __forceinline__ void sum_stride(const float* __restrict__ y, int64_t lo, int64_t hi,
                                           int t, int P, ff_t& acc) {
    constexpr int U = 8;
    int64_t i = lo + t;
    for (; i + (int64_t)(U - 1) * P < hi; i += (int64_t)U * P) {
        float r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = y[i + (int64_t)u * P];
#pragma unroll
        for (int u = 0; u < U; ++u) comp_add(acc, r[u]);
    }
    for (; i < hi; i += P) comp_add(acc, y[i]);
}

// MODE 1: the lane runs of the first lw1 (loop 1) / lw2 (loop 2) waves of a
// team go through a per-wave LDS buffer (lines.h; 16 KiB a wave of dynamic
// shared memory); MODE 2: short runs as the union of the wave's runs in both
// loops.  With nowait both loops have the same schedule, so lw1 == lw2 and a
// wave splits every run the same way in both: the lane that loads a 16-byte
// block of y in loop 2 is the lane that stored it in loop 1 (the two loops
// also take the lines in the same order: line_rot depends only on the wave
// and the run's line count), and the heads and tails of the runs stay with
// their owners.
template <bool NOWAIT, int MODE>
__global__ __launch_bounds__(MODE ? 512 : 1024) void region_axpy_then_sum_kernel(
    float a, const float* __restrict__ x, float* __restrict__ y, float* __restrict__ sum,
    int64_t n, int P, int64_t dc, int64_t c1, int64_t c2, int lw1, int lw2, CrossTeam ct) {
    using R = Red<DT_F32, OP_SUM>;
    using R1 = CompSum<float, 1>;
    extern __shared__ f32x4 stage[];
    __shared__ ff_t lds_slots[kMaxWaves];
    __shared__ int s_last;
    const int64_t T = gridDim.x, k = blockIdx.x;
    const int t = threadIdx.x;
    const int wave = t / kWave;
    const uint32_t epoch = T > 1 ? read_epoch(ct.epoch) : 0u;
    const int64_t nb = team_nblocks(n, T, dc, k);
    f32x4* xs = stage + (size_t)wave * (2 * kStageSlots);
    f32x4* ys = xs + kStageSlots;
    // loop 1: the AXPY update (its sum is not used here)
    if (t < P) {
        ff_t unused = R::identity();
        for (int64_t b = 0; b < nb; ++b) {
            const Range blk = team_block(n, T, dc, k, b);
            const int64_t m = blk.hi - blk.lo;
            if (c1 == 1) {
                axpy_stride(a, x, y, blk.lo, blk.hi, t, P, unused);
                continue;
            }
            const int64_t nc = thread_nchunks(m, P, c1, t);
            int64_t j = 0;
            if (MODE && wave < lw1) {
                const int64_t full = c1 == 0 ? 1 : thread_nchunks(m, P, c1, t | (kWave - 1));
                for (; j < full; ++j) {
                    const Range ch = thread_chunk(blk.lo, m, P, c1, t, j);
                    if (MODE == 2)
                        axpy_run_union(a, x, y, ch.lo, ch.hi, xs, ys, unused);
                    else
                        axpy_run_lines(a, x, y, ch.lo, ch.hi, xs, ys, unused);
                }
            }
            for (; j < nc; ++j) {
                const Range ch = thread_chunk(blk.lo, m, P, c1, t, j);
                if (c1 > 16 || !axpy_short_run(a, x, y, ch.lo, ch.hi, unused))
                    axpy_range(a, x, y, ch.lo, ch.hi, unused);
            }
        }
    }
    if constexpr (!NOWAIT) __syncthreads();   // loop 1's implicit barrier
    // loop 2: reduction(+: s) over the updated y
    ff_t acc = R::identity();
    if (t < P) {
        for (int64_t b = 0; b < nb; ++b) {
            const Range blk = team_block(n, T, dc, k, b);
            const int64_t m = blk.hi - blk.lo;
            if (c2 == 1) {
                sum_stride(y, blk.lo, blk.hi, t, P, acc);
                continue;
            }
            const int64_t nc = thread_nchunks(m, P, c2, t);
            int64_t j = 0;
            if (MODE == 2 && wave < lw2) {
                const int64_t full = c2 == 0 ? 1 : thread_nchunks(m, P, c2, t | (kWave - 1));
                for (; j < full; ++j) {
                    const Range ch = thread_chunk(blk.lo, m, P, c2, t, j);
                    sum_run_union(y, ch.lo, ch.hi, xs, ys, acc);
                }
            } else if (MODE == 1 && wave < lw2) {
                const int64_t full = c2 == 0 ? 1 : thread_nchunks(m, P, c2, t | (kWave - 1));
                for (; j < full; ++j) {
                    const Range ch = thread_chunk(blk.lo, m, P, c2, t, j);
                    int64_t l0, np;
                    run_lines<4>(y, ch.lo, ch.hi, l0, np);
                    if (l0 > ch.lo) sum_range(y, ch.lo, l0, acc);
                    line_fold<R1, DT_F32>(y, l0, np, reinterpret_cast<u32x4*>(xs), &acc);
                    const int64_t r = l0 + np * (kLineBytes / 4);
                    if (r < ch.hi) sum_range(y, r, ch.hi, acc);
                }
            }
            for (; j < nc; ++j) {
                const Range ch = thread_chunk(blk.lo, m, P, c2, t, j);
                sum_range(y, ch.lo, ch.hi, acc);
            }
        }
    }
    axpy_finish_sum(acc, sum, ct, epoch, lds_slots, &s_last);
}

template <bool NOWAIT>
static hipError_t launch_region(float a, const float* x, float* y, float* sum, int64_t n,
                                int teams, int threads, int64_t dc, int64_t c1, int64_t c2,
                                const CrossTeam& ct, hipStream_t stream) {
    constexpr int64_t kMinChunk = 64;
    constexpr int64_t kUnionMinChunk = 16;
    const int block = (threads + kWave - 1) / kWave * kWave;
    const bool co_aligned =
        ((reinterpret_cast<uintptr_t>(x) ^ reinterpret_cast<uintptr_t>(y)) & 15) == 0;
    // Short runs off the line grid (both loops) as the union of the wave's
    // runs, whole-line runs through the lane-run lines, as for the AXPY body
    // alone.
    const int64_t m_hi = dc ? std::min<int64_t>(dc, n) : (n + teams - 1) / teams;
    const bool blocks_on_grid = (reinterpret_cast<uintptr_t>(y) & (kLineBytes - 1)) == 0 &&
                                (dc ? dc % 32 == 0 : n % teams == 0 && (n / teams) % 32 == 0);
    auto whole = [&](int64_t c) {
        return blocks_on_grid && (c > 0 ? c % 32 == 0
                                        : (n / teams) % threads == 0 &&
                                              (n / teams / threads) % 32 == 0);
    };
    // (runs of up to 64: longer ones, e.g. chunk 100, ran slower through the
    // union in the two-loop region, 4.47 -> 3.83 TB/s)
    constexpr int64_t kRegionUnionRun = 64;
    auto short_runs = [&](int64_t c) {
        return c > 0 ? c >= kUnionMinChunk && c <= kRegionUnionRun
                     : (m_hi + threads - 1) / threads <= kRegionUnionRun;
    };
    int lw1 = co_aligned ? lines_waves(n, teams, threads, dc, c1, 4, kMinChunk, 512) : 0;
    int lw2 = lines_waves(n, teams, threads, dc, c2, 4, kMinChunk, 512);
    if (NOWAIT) lw1 = lw2 = std::min(lw1, lw2);   // the same split of every run in both loops
    int mode = std::max(lw1, lw2) ? 1 : 0;
    const bool lines_whole = lw1 && lw2 && whole(c1) && whole(c2);
    if (!lines_whole && co_aligned && threads % kWave == 0 && threads <= 512 && n > 0 &&
        short_runs(c1) && short_runs(c2) && c1 != 1 && c2 != 1) {
        mode = 2;
        auto uw = [&](int64_t c) {
            return c > 0 ? lines_waves(n, teams, threads, dc, c, 4, kUnionMinChunk, 512)
                         : threads / kWave;
        };
        lw1 = uw(c1);
        lw2 = uw(c2);
        if (NOWAIT) lw1 = lw2 = std::min(lw1, lw2);
        if (std::max(lw1, lw2) == 0) mode = 0;
    }
    if (mode == 0) {
        hipLaunchKernelGGL((region_axpy_then_sum_kernel<NOWAIT, 0>), dim3(teams), dim3(block), 0,
                           stream, a, x, y, sum, n, threads, dc, c1, c2, 0, 0, ct);
        return hipGetLastError();
    }
    const size_t lds = (size_t)std::max(lw1, lw2) * 2 * kStageSlots * 16;
    const void* fn = mode == 2
                         ? reinterpret_cast<const void*>(region_axpy_then_sum_kernel<NOWAIT, 2>)
                         : reinterpret_cast<const void*>(region_axpy_then_sum_kernel<NOWAIT, 1>);
    if (lds > 64 * 1024) {   // past the default dynamic LDS limit: ask for it
        const hipError_t attr =
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (attr != hipSuccess) return attr;
    }
    if (mode == 2)
        hipLaunchKernelGGL((region_axpy_then_sum_kernel<NOWAIT, 2>), dim3(teams), dim3(block),
                           lds, stream, a, x, y, sum, n, threads, dc, c1, c2, lw1, lw2, ct);
    else
        hipLaunchKernelGGL((region_axpy_then_sum_kernel<NOWAIT, 1>), dim3(teams), dim3(block),
                           lds, stream, a, x, y, sum, n, threads, dc, c1, c2, lw1, lw2, ct);
    return hipGetLastError();
}

}  // namespace omprt

using namespace omprt;

extern "C" omprt_status omprt_region_axpy_sum(float a, const float* d_x, float* d_y, float* d_sum,
                                              const omprt_sched* s, int64_t chunk2,
                                              int32_t nowait, const omprt_config* cfg,
                                              void* hip_stream) {
    if (omprt_status st = check_sched(s, true)) return st;
    if (chunk2 < 0) return fail(OMPRT_ERR_INVALID, "chunk2 %lld < 0", (long long)chunk2);
    if (nowait && chunk2 != s->chunk)
        return fail(OMPRT_ERR_INVALID,
                    "nowait needs the same static schedule in both loops (chunk %lld vs %lld): "
                    "otherwise loop 2 reads elements another thread of loop 1 writes",
                    (long long)s->chunk, (long long)chunk2);
    if (!d_sum) return fail(OMPRT_ERR_INVALID, "sum is NULL");
    if (s->n > 0 && (!d_x || !d_y)) return fail(OMPRT_ERR_INVALID, "x/y is NULL with n > 0");
    if ((reinterpret_cast<uintptr_t>(d_x) | reinterpret_cast<uintptr_t>(d_y) |
         reinterpret_cast<uintptr_t>(d_sum)) % 4)
        return fail(OMPRT_ERR_INVALID, "x, y or sum not aligned to 4 bytes");
    if (s->n > 0) {
        const char* xb = reinterpret_cast<const char*>(d_x);
        const char* yb = reinterpret_cast<const char*>(d_y);
        if (xb < yb + s->n * 4 && yb < xb + s->n * 4) return fail(OMPRT_ERR_INVALID, "x and y overlap");
    }
    LaunchCfg lc;
    // body 2: the AXPY-then-sum region (the AXPY body's model features, its own heuristic)
    if (omprt_status st = resolve_config(s->n, OMPRT_F32, OMPRT_SUM, 2, s->chunk, cfg, &lc, nullptr))
        return st;
    const int teams = s->num_teams ? s->num_teams : lc.teams;
    if (teams > 65535)
        return fail(OMPRT_ERR_INVALID, "num_teams %d above 65535 (cross-team slot limit)", teams);
    const int threads = s->threads_per_team ? s->threads_per_team : lc.threads;
    if (s->n == 0) return OMPRT_OK;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    Workspace* ws = nullptr;
    if (omprt_status st = workspace_get(stream, teams, &ws)) return st;
    const CrossTeamArgs ca = ws->cross();
    const CrossTeam ct{static_cast<uint64_t*>(ca.slots), ca.counter, ca.epoch, ca.status};
    const hipError_t e =
        nowait ? launch_region<true>(a, d_x, d_y, d_sum, s->n, teams, threads, s->dist_chunk,
                                     s->chunk, chunk2, ct, stream)
               : launch_region<false>(a, d_x, d_y, d_sum, s->n, teams, threads, s->dist_chunk,
                                      s->chunk, chunk2, ct, stream);
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "region launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}
