// map_axpy.hip -- kernels that execute a loop body under the exact static
// schedule: every iteration runs on the thread the schedule assigns it to.
//
// static_map_kernel records the mapping itself (owner id, execution count);
// axpy_sum_kernel runs y[i] <- fmaf(a, x[i], y[i]) and reduces the updated
// y with a compensated sum through the same team tree and last-team
// combine as the plain reduction.
#include "axpy.h"
#include "device.h"
#include "launch.h"

namespace omprt {

// ---------------------------------------------------------------- iteration map

__global__ __launch_bounds__(1024) void static_map_kernel(int64_t n, int P, int64_t dc,
                                                          int64_t c, int32_t* __restrict__ owner,
                                                          uint32_t* __restrict__ count) {
    const int64_t T = gridDim.x, k = blockIdx.x;
    const int t = threadIdx.x;
    if (t >= P) return;   // lanes beyond the logical team size
    const int32_t id = (int32_t)(k * P + t);
    const int64_t nb = team_nblocks(n, T, dc, k);
    for (int64_t i = 0; i < nb; ++i) {
        const Range blk = team_block(n, T, dc, k, i);
        const int64_t m = blk.hi - blk.lo;
        const int64_t nc = thread_nchunks(m, P, c, t);
        for (int64_t j = 0; j < nc; ++j) {
            const Range ch = thread_chunk(blk.lo, m, P, c, t, j);
            for (int64_t it = ch.lo; it < ch.hi; ++it) {
                owner[it] = id;
                atomicAdd(count + it, 1u);
            }
        }
    }
}

hipError_t launch_static_map(int64_t n, int teams, int threads, int64_t dist_chunk,
                             int64_t chunk, int32_t* owner, uint32_t* count,
                             hipStream_t stream) {
    const int block = (threads + kWave - 1) / kWave * kWave;
    hipLaunchKernelGGL(static_map_kernel, dim3(teams), dim3(block), 0, stream, n, threads,
                       dist_chunk, chunk, owner, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------- AXPY + sum

// MODE 1: lane runs (chunk 0, or chunks of at least kLinesMinChunk) of the
// first `lw` waves of a team go through a per-wave LDS buffer of 2 x 8 KiB
// (x lines, y lines) in dynamic shared memory, each lane's run a line per
// pass; MODE 2: short runs (chunks of kUnionMinChunk to kUnionRun
// iterations, or chunk 0 with at most kUnionRun a lane) go through the same
// buffer as the union of the wave's side-by-side runs.  The host takes them
// when the team is whole waves and x and y are co-aligned to 16 bytes, and
// sizes lw to the waves that can have a chunk at all (later waves' lanes
// get none); MODE 0 runs every lane alone.
constexpr int64_t kLinesMinChunk = 64;
constexpr int64_t kUnionMinChunk = 16;
constexpr int kLinesWaveBytes = 2 * kStageSlots * 16;

template <int MODE>
__global__ __launch_bounds__(MODE ? 512 : 1024) void axpy_sum_kernel(
    float a, const float* __restrict__ x, float* __restrict__ y, float* __restrict__ sum,
    int64_t n, int P, int64_t dc, int64_t c, int lw, CrossTeam ct) {
    using R = Red<DT_F32, OP_SUM>;
    extern __shared__ f32x4 stage[];
    __shared__ ff_t lds_slots[kMaxWaves];
    __shared__ int s_last;
    const int64_t T = gridDim.x, k = blockIdx.x;
    const int t = threadIdx.x;
    const uint32_t epoch = T > 1 ? read_epoch(ct.epoch) : 0u;
    ff_t acc = R::identity();
    if (t < P) {
        f32x4* xs = stage + (size_t)(t / kWave) * (2 * kStageSlots);
        f32x4* ys = xs + kStageSlots;
        const int64_t nb = team_nblocks(n, T, dc, k);
        for (int64_t i = 0; i < nb; ++i) {
            const Range blk = team_block(n, T, dc, k, i);
            const int64_t m = blk.hi - blk.lo;
            if (c == 1) {   // the same iterations as the chunk loop below, strided
                axpy_stride(a, x, y, blk.lo, blk.hi, t, P, acc);
                continue;
            }
            const int64_t nc = thread_nchunks(m, P, c, t);
            int64_t j = 0;
            if (MODE && t / kWave < lw) {
                // Rounds in which every lane of the wave has a chunk (chunk
                // counts do not grow with the thread number, so the wave's
                // last lane has the fewest) run through LDS.
                const int64_t full = c == 0 ? 1 : thread_nchunks(m, P, c, t | (kWave - 1));
                for (; j < full; ++j) {
                    const Range ch = thread_chunk(blk.lo, m, P, c, t, j);
                    if (MODE == 2)
                        axpy_run_union(a, x, y, ch.lo, ch.hi, xs, ys, acc);
                    else
                        axpy_run_lines(a, x, y, ch.lo, ch.hi, xs, ys, acc);
                }
            }
            for (; j < nc; ++j) {
                const Range ch = thread_chunk(blk.lo, m, P, c, t, j);
                if (c > 16 || !axpy_short_run(a, x, y, ch.lo, ch.hi, acc))
                    axpy_range(a, x, y, ch.lo, ch.hi, acc);
            }
        }
    }
    axpy_finish_sum(acc, sum, ct, epoch, lds_slots, &s_last);
}

hipError_t launch_axpy_sum(float a, const float* x, float* y, float* sum, int64_t n, int teams,
                           int threads, int64_t dist_chunk, int64_t chunk, const CrossTeamArgs& ct,
                           hipStream_t stream) {
    const int block = (threads + kWave - 1) / kWave * kWave;
    const CrossTeam dct{static_cast<uint64_t*>(ct.slots), ct.counter, ct.epoch, ct.status};
    const bool co_aligned =
        ((reinterpret_cast<uintptr_t>(x) ^ reinterpret_cast<uintptr_t>(y)) & 15) == 0;
    const bool waves = threads % kWave == 0 && threads <= 512;
    // Whole-line runs (every lane's runs start on a 128-byte line of y and
    // cover whole lines: the team blocks and the chunk, or chunk 0's equal
    // shares, multiples of 32 elements) take the lane-run lines; other runs
    // of 16 to kUnionRun elements take the union of the wave's runs, which
    // has no per-lane edges.  2^26 fp32 on gfx950, chunk 64 with team blocks
    // off the line grid: 3.22 -> 4.62 TB/s; chunk 32: 3.92 -> 5.10; chunk 0
    // with 32-element shares off the grid: 1.79 -> 3.83; whole-line runs
    // keep the lane-run lines (chunk 0 with 128-element shares: 5.25 against
    // 4.61 through the union).
    const int64_t m_hi = dist_chunk ? std::min<int64_t>(dist_chunk, n) : (n + teams - 1) / teams;
    const bool blocks_on_grid = (reinterpret_cast<uintptr_t>(y) & (kLineBytes - 1)) == 0 &&
                                (dist_chunk ? dist_chunk % 32 == 0
                                            : n % teams == 0 && (n / teams) % 32 == 0);
    const bool whole_runs =
        blocks_on_grid && (chunk > 0 ? chunk % 32 == 0
                                     : (n / teams) % threads == 0 && (n / teams / threads) % 32 == 0);
    // off the grid from chunk 8 (2^26: chunk 8 1.90 -> 2.95 TB/s, 12 2.46 ->
    // 3.96, 15 2.39 -> 4.32); on the grid chunks of 4 to 16 that are whole
    // vectors take axpy_short_run instead
    const int64_t union_min = blocks_on_grid ? kUnionMinChunk : 8;
    const bool short_runs = chunk > 0 ? chunk >= union_min && chunk <= kUnionRun
                                      : (m_hi + threads - 1) / threads <= kUnionRun;
    int mode = 0, lw = 0;
    const int lw_lines =
        co_aligned ? lines_waves(n, teams, threads, dist_chunk, chunk, 4, kLinesMinChunk, 512) : 0;
    if (lw_lines && whole_runs) {
        mode = 1;
        lw = lw_lines;
    } else if (co_aligned && waves && n > 0 && short_runs) {
        mode = 2;
        lw = chunk > 0 ? lines_waves(n, teams, threads, dist_chunk, chunk, 4, union_min, 512)
                       : threads / kWave;
    } else if (lw_lines) {
        mode = 1;
        lw = lw_lines;
    }
    if (mode == 0 || lw == 0) {
        hipLaunchKernelGGL(axpy_sum_kernel<0>, dim3(teams), dim3(block), 0, stream, a, x, y, sum,
                           n, threads, dist_chunk, chunk, 0, dct);
        return hipGetLastError();
    }
    const size_t lds = (size_t)lw * kLinesWaveBytes;
    const void* fn = mode == 2 ? reinterpret_cast<const void*>(axpy_sum_kernel<2>)
                               : reinterpret_cast<const void*>(axpy_sum_kernel<1>);
    if (lds > 64 * 1024) {   // past the default dynamic LDS limit: ask for it
        const hipError_t attr =
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (attr != hipSuccess) return attr;
    }
    if (mode == 2)
        hipLaunchKernelGGL(axpy_sum_kernel<2>, dim3(teams), dim3(block), lds, stream, a, x, y, sum,
                           n, threads, dist_chunk, chunk, lw, dct);
    else
        hipLaunchKernelGGL(axpy_sum_kernel<1>, dim3(teams), dim3(block), lds, stream, a, x, y, sum,
                           n, threads, dist_chunk, chunk, lw, dct);
    return hipGetLastError();
}

}  // namespace omprt
