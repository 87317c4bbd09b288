// generic.hip -- a target region in generic (non-SPMD) mode: one team whose
// main thread (thread 0) runs the region's sequential code and hands each
// parallel loop to the team through a work descriptor in team-shared memory
// (the routines a compiled target region calls, paper sec. 2.1).  The other
// threads wait at the team barrier for work -- a state machine -- run their
// share of the loop and meet the main thread, which works on the loop as
// thread 0 of the team, at the join barrier.  One launch runs the whole
// region, however many parallel loops it has, so nothing returns to the
// host between them.
//
// The region is a power iteration on a diagonal matrix D = diag(d):
//   repeat iters times:
//     parallel loop:   w = d * v (written over v), s = sum of w^2
//     sequential code: r = 1 / sqrt(s)
//     parallel loop:   v = w * r
//   sequential code:   lambda = sqrt(s)
// Loops take the static schedule with chunk 1 (thread t owns iterations
// t, t + P, ...), so a wave's lanes touch neighbouring elements and every
// thread rewrites in the second loop exactly the elements it wrote in the
// first.  s accumulates in compensated fp32 (TwoSum per element,
// float-float through the team tree).
#include "device.h"
#include "runtime.h"

namespace omprt {

enum { WORK_EXIT = 0, WORK_SCALE_SQUARES = 1, WORK_NORMALISE = 2 };

constexpr int kGenericUnroll = 8;   // loads in flight per lane and array

__device__ __forceinline__ void loop_scale_squares(const float* __restrict__ d,
                                                   float* __restrict__ v, int64_t n, ff_t& acc) {
    constexpr int U = kGenericUnroll;
    const int64_t P = blockDim.x;
    int64_t i = threadIdx.x;
    for (; i + (U - 1) * P < n; i += U * P) {
        float a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = d[i + u * P];
            b[u] = v[i + u * P];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float w = a[u] * b[u];
            v[i + u * P] = w;
            comp_add(acc, w * w);
        }
    }
    for (; i < n; i += P) {
        const float w = d[i] * v[i];
        v[i] = w;
        comp_add(acc, w * w);
    }
}

__device__ __forceinline__ void loop_normalise(float* __restrict__ v, int64_t n, float r) {
    constexpr int U = kGenericUnroll;
    const int64_t P = blockDim.x;
    int64_t i = threadIdx.x;
    for (; i + (U - 1) * P < n; i += U * P) {
        float b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) b[u] = v[i + u * P];
#pragma unroll
        for (int u = 0; u < U; ++u) v[i + u * P] = b[u] * r;
    }
    for (; i < n; i += P) v[i] *= r;
}

__global__ __launch_bounds__(1024) void generic_power_kernel(const float* __restrict__ d,
                                                             float* __restrict__ v, int64_t n,
                                                             int iters, float* __restrict__ lambda) {
    using R = Red<DT_F32, OP_SUM>;
    __shared__ int s_work;       // the work descriptor: which loop runs next
    __shared__ float s_scale;    // and its argument
    __shared__ ff_t s_red[kMaxWaves];
    __shared__ ff_t s_sum;       // result of the last reduction loop
    const int tid = threadIdx.x;
    // the main thread's sequential state (only thread 0's copy is used)
    int k = 0;
    int last = WORK_EXIT;
    float s = 0.0f;
    for (;;) {
        if (tid == 0) {   // sequential code
            if (last == WORK_SCALE_SQUARES) {
                s = s_sum.hi + s_sum.lo;
                s_scale = 1.0f / sqrtf(s);
                s_work = WORK_NORMALISE;
            } else {
                if (last == WORK_NORMALISE) ++k;
                if (k == iters) {
                    lambda[0] = sqrtf(s);
                    s_work = WORK_EXIT;
                } else {
                    s_work = WORK_SCALE_SQUARES;
                }
            }
        }
        __syncthreads();   // the team picks up the work descriptor
        const int work = s_work;
        if (work == WORK_EXIT) break;
        if (work == WORK_SCALE_SQUARES) {
            ff_t acc = R::identity();
            loop_scale_squares(d, v, n, acc);
            acc = team_reduce<R>(acc, s_red);
            if (tid == 0) s_sum = acc;
        } else {
            loop_normalise(v, n, s_scale);
        }
        __syncthreads();   // join: the loop is complete and its writes visible
        last = work;
    }
}

}  // namespace omprt

using namespace omprt;

extern "C" omprt_status omprt_generic_power(const float* d_diag, float* d_v, int64_t n,
                                            int32_t iters, int32_t threads, float* d_lambda,
                                            void* hip_stream) {
    if (n < 1 || n > ((int64_t)1 << 32))
        return fail(OMPRT_ERR_INVALID, "n = %lld outside 1..2^32", (long long)n);
    if (iters < 1) return fail(OMPRT_ERR_INVALID, "iters %d < 1", iters);
    if (threads == 0) threads = 1024;
    if (threads < 64 || threads > 1024 || threads % 64)
        return fail(OMPRT_ERR_INVALID, "threads %d: 64..1024, a multiple of 64", threads);
    if (!d_diag || !d_v || !d_lambda) return fail(OMPRT_ERR_INVALID, "NULL pointer");
    if ((reinterpret_cast<uintptr_t>(d_diag) | reinterpret_cast<uintptr_t>(d_v) |
         reinterpret_cast<uintptr_t>(d_lambda)) % sizeof(float))
        return fail(OMPRT_ERR_INVALID, "pointer not aligned to 4 bytes");
    const uintptr_t db = reinterpret_cast<uintptr_t>(d_diag), vb = reinterpret_cast<uintptr_t>(d_v),
                    lb = reinterpret_cast<uintptr_t>(d_lambda), nb = (uintptr_t)n * sizeof(float);
    if (db < vb + nb && vb < db + nb) return fail(OMPRT_ERR_INVALID, "diag and v overlap");
    if ((lb >= vb && lb < vb + nb) || (lb >= db && lb < db + nb))
        return fail(OMPRT_ERR_INVALID, "lambda lies inside diag or v");
    hipLaunchKernelGGL(generic_power_kernel, dim3(1), dim3(threads), 0,
                       static_cast<hipStream_t>(hip_stream), d_diag, d_v, n, (int)iters, d_lambda);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "generic launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}
