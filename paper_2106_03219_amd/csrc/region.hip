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

// LINES: the lane runs of the first lw1 (loop 1) / lw2 (loop 2) waves of a
// team go through a per-wave LDS buffer (lines.h; 16 KiB a wave of dynamic
// shared memory).  With nowait both loops have the same schedule, so lw1 ==
// lw2 and a wave splits every run the same way in both: the lane that loads
// a 16-byte block of y in loop 2 is the lane that stored it in loop 1, and
// the heads and tails of the runs stay with their owners.
template <bool NOWAIT, bool LINES>
__global__ __launch_bounds__(LINES ? 512 : 1024) void region_axpy_then_sum_kernel(
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
            if (LINES && wave < lw1) {
                const int64_t full = c1 == 0 ? 1 : thread_nchunks(m, P, c1, t | (kWave - 1));
                for (; j < full; ++j) {
                    const Range ch = thread_chunk(blk.lo, m, P, c1, t, j);
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
            if (LINES && wave < lw2) {
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
    const int block = (threads + kWave - 1) / kWave * kWave;
    const bool co_aligned =
        ((reinterpret_cast<uintptr_t>(x) ^ reinterpret_cast<uintptr_t>(y)) & 15) == 0;
    int lw1 = co_aligned ? lines_waves(n, teams, threads, dc, c1, 4, kMinChunk, 512) : 0;
    int lw2 = lines_waves(n, teams, threads, dc, c2, 4, kMinChunk, 512);
    if (NOWAIT) lw1 = lw2 = std::min(lw1, lw2);   // the same split of every run in both loops
    const int lw = std::max(lw1, lw2);
    if (lw == 0) {
        hipLaunchKernelGGL((region_axpy_then_sum_kernel<NOWAIT, false>), dim3(teams), dim3(block),
                           0, stream, a, x, y, sum, n, threads, dc, c1, c2, 0, 0, ct);
        return hipGetLastError();
    }
    const size_t lds = (size_t)lw * 2 * kStageSlots * 16;
    if (lds > 64 * 1024) {   // past the default dynamic LDS limit: ask for it
        const hipError_t attr = hipFuncSetAttribute(
            reinterpret_cast<const void*>(region_axpy_then_sum_kernel<NOWAIT, true>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (attr != hipSuccess) return attr;
    }
    hipLaunchKernelGGL((region_axpy_then_sum_kernel<NOWAIT, true>), dim3(teams), dim3(block), lds,
                       stream, a, x, y, sum, n, threads, dc, c1, c2, lw1, lw2, ct);
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
