// map_axpy.hip -- kernels that execute a loop body under the exact static
// schedule: every iteration runs on the thread the schedule assigns it to.
//
// static_map_kernel records the mapping itself (owner id, execution count);
// axpy_sum_kernel runs y[i] <- fmaf(a, x[i], y[i]) and reduces the updated
// y with a compensated sum through the same team tree and last-team
// combine as the plain reduction.
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

__device__ __forceinline__ void axpy_elem(float a, const float* __restrict__ x,
                                          float* __restrict__ y, int64_t i, ff_t& acc) {
    const float r = __builtin_fmaf(a, x[i], y[i]);
    y[i] = r;
    comp_add(acc, r);
}

// One chunk [lo, hi) of the calling thread, 16-byte vectors where x and y
// are co-aligned.
__device__ __forceinline__ void axpy_range(float a, const float* __restrict__ x,
                                           float* __restrict__ y, int64_t lo, int64_t hi,
                                           ff_t& acc) {
    const bool co_aligned =
        ((reinterpret_cast<uintptr_t>(x) ^ reinterpret_cast<uintptr_t>(y)) & 15) == 0;
    if (!co_aligned || hi - lo < 8) {
        for (int64_t i = lo; i < hi; ++i) axpy_elem(a, x, y, i, acc);
        return;
    }
    const uintptr_t mis = reinterpret_cast<uintptr_t>(y + lo) & 15;
    const int64_t head = (int64_t)(((16 - mis) & 15) / 4);
    for (int64_t i = lo; i < lo + head; ++i) axpy_elem(a, x, y, i, acc);
    const int64_t p = lo + head;
    const int64_t nv = (hi - p) / 4;
    const float4* __restrict__ xv = reinterpret_cast<const float4*>(x + p);
    float4* __restrict__ yv = reinterpret_cast<float4*>(y + p);
    // eight 16-byte vectors of x and of y in flight per lane -- a whole 128-byte
    // line of each -- so a lane's loads to one line issue together and the
    // line is fetched once (measured at 2^26, chunk 0: 4.26 TB/s with eight,
    // 3.65 with four, 2.91 with sixteen)
    constexpr int U = 8;
    int64_t j = 0;
    for (; j + U <= nv; j += U) {
        float4 xx[U], yy[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xx[u] = xv[j + u];
            yy[u] = yv[j + u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            yy[u].x = __builtin_fmaf(a, xx[u].x, yy[u].x);
            yy[u].y = __builtin_fmaf(a, xx[u].y, yy[u].y);
            yy[u].z = __builtin_fmaf(a, xx[u].z, yy[u].z);
            yy[u].w = __builtin_fmaf(a, xx[u].w, yy[u].w);
            yv[j + u] = yy[u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            comp_add(acc, yy[u].x);
            comp_add(acc, yy[u].y);
            comp_add(acc, yy[u].z);
            comp_add(acc, yy[u].w);
        }
    }
    for (; j < nv; ++j) {
        const float4 xx = xv[j];
        float4 yy = yv[j];
        yy.x = __builtin_fmaf(a, xx.x, yy.x);
        yy.y = __builtin_fmaf(a, xx.y, yy.y);
        yy.z = __builtin_fmaf(a, xx.z, yy.z);
        yy.w = __builtin_fmaf(a, xx.w, yy.w);
        yv[j] = yy;
        comp_add(acc, yy.x);
        comp_add(acc, yy.y);
        comp_add(acc, yy.z);
        comp_add(acc, yy.w);
    }
    for (int64_t i = p + nv * 4; i < hi; ++i) axpy_elem(a, x, y, i, acc);
}

// Chunk size 1: thread t of the block [lo, hi) executes lo + t, lo + t + P,
// ... (one-iteration chunks dealt round-robin).  A wave's lanes touch 64
// consecutive elements, so every access is coalesced and covers whole cache
// lines: the streams bypass cache residency (nontemporal), four rows in
// flight.  (Nontemporal access is a loss for the per-lane runs of larger
// chunks, whose lines are consumed by several successive loads.)
__device__ __forceinline__ void axpy_stride(float a, const float* __restrict__ x,
                                            float* __restrict__ y, int64_t lo, int64_t hi,
                                            int t, int P, ff_t& acc) {
    constexpr int U = 4;
    int64_t i = lo + t;
    for (; i + (int64_t)(U - 1) * P < hi; i += (int64_t)U * P) {
        float xx[U], yy[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xx[u] = __builtin_nontemporal_load(x + i + (int64_t)u * P);
            yy[u] = __builtin_nontemporal_load(y + i + (int64_t)u * P);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            yy[u] = __builtin_fmaf(a, xx[u], yy[u]);
            __builtin_nontemporal_store(yy[u], y + i + (int64_t)u * P);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) comp_add(acc, yy[u]);
    }
    for (; i < hi; i += P) axpy_elem(a, x, y, i, acc);
}

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
                axpy_range(a, x, y, ch.lo, ch.hi, acc);
            }
        }
    }
    acc = team_reduce<R>(acc, lds_slots);
    if (T == 1) {
        if (t == 0) sum[0] = R::finish(acc, sum[0]);
        return;
    }
    const uint32_t tag = launch_tag(epoch);
    if (!publish_and_elect(acc, ct.slots + (size_t)k * kSlotWords, ct.counter, (uint32_t)(T - 1),
                           tag, &s_last))
        return;
    const ff_t cmb = combine_slots<R>(ct.slots, T, tag, ct.status, lds_slots);
    if (t == 0) {
        sum[0] = R::finish(cmb, sum[0]);
        advance_epoch(ct.epoch, epoch);
    }
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
