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

__global__ __launch_bounds__(1024) void axpy_sum_kernel(float a, const float* __restrict__ x,
                                                        float* __restrict__ y,
                                                        float* __restrict__ sum, int64_t n, int P,
                                                        int64_t dc, int64_t c, CrossTeam ct) {
    using R = Red<DT_F32, OP_SUM>;
    __shared__ ff_t lds_slots[kMaxWaves];
    __shared__ int s_last;
    const int64_t T = gridDim.x, k = blockIdx.x;
    const int t = threadIdx.x;
    const uint32_t epoch = T > 1 ? read_epoch(ct.epoch) : 0u;
    ff_t acc = R::identity();
    if (t < P) {
        const int64_t nb = team_nblocks(n, T, dc, k);
        for (int64_t i = 0; i < nb; ++i) {
            const Range blk = team_block(n, T, dc, k, i);
            const int64_t m = blk.hi - blk.lo;
            if (c == 1) {   // the same iterations as the chunk loop below, strided
                axpy_stride(a, x, y, blk.lo, blk.hi, t, P, acc);
                continue;
            }
            const int64_t nc = thread_nchunks(m, P, c, t);
            for (int64_t j = 0; j < nc; ++j) {
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
    hipLaunchKernelGGL(axpy_sum_kernel, dim3(teams), dim3(block), 0, stream, a, x, y, sum, n,
                       threads, dist_chunk, chunk, dct);
    return hipGetLastError();
}

}  // namespace omprt
