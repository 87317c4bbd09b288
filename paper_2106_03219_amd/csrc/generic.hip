// generic.hip -- a target region in generic (non-SPMD) mode: each team's
// main thread (thread 0) runs the region's sequential code and hands each
// parallel loop to its team through a work descriptor in team-shared
// memory (the routines a compiled target region calls, paper sec. 2.1).
// The other threads wait at the team barrier for work -- a state machine --
// run their share of the loop and meet the main thread, which works on the
// loop as thread 0 of the team, at the join barrier.  One launch runs the
// whole region, however many parallel loops it has, so nothing returns to
// the host between them.
//
// The region is a power iteration on a diagonal matrix D = diag(d):
//   repeat iters times:
//     parallel loop:   w = d * v (written over v), s = sum of w^2
//     sequential code: r = 1 / sqrt(s)
//     parallel loop:   v = w * r
//   sequential code:   lambda = sqrt(s)
// s accumulates in compensated fp32 (TwoSum per element, float-float
// through the team tree).
//
// With one team (the mode's own shape) the team owns [0, n).  With T > 1
// co-resident teams the loops are also distributed: team k owns the
// balanced block bal(n, T, k) in both loops, every team runs the
// sequential code on the same values, and the sum reaches all of them by an
// all-gather of team partials: each team publishes its partial as tagged
// slot words (the cross-team slots of the reductions; tag = the launch tag
// of epoch + step), then reads every team's partial in team order, so all
// teams hold bit-identical s.  Steps alternate between two slot sets: a
// team can run at most one step ahead of another (step k + 1's all-gather
// needs everyone's step k + 1 partial), so a set is overwritten only after
// every team has read it.  The normalising loop touches only the team's own
// block, so it needs no cross-team wait.  Inside a team loops take the
// static schedule with chunk 1 (thread t owns lo + t, lo + t + P, ...), so
// a wave's lanes touch neighbouring elements and each thread rewrites in
// the second loop exactly the elements it wrote in the first.
#include <algorithm>

#include "device.h"
#include "runtime.h"
#include "sched.h"

namespace omprt {

enum { WORK_EXIT = 0, WORK_SCALE_SQUARES = 1, WORK_NORMALISE = 2 };

constexpr int kGenericUnroll = 8;   // loads in flight per lane and array
// Teams of the distributed form: each team reads every team's partial once a
// step, so the all-gather grows as teams^2 (512 teams: 4 MiB of L2 reads).
constexpr int kMaxGenericTeams = 512;

__device__ __forceinline__ void loop_scale_squares(const float* __restrict__ d,
                                                   float* __restrict__ v, int64_t lo, int64_t hi,
                                                   ff_t& acc) {
    constexpr int U = kGenericUnroll;
    const int64_t P = blockDim.x;
    int64_t i = lo + threadIdx.x;
    for (; i + (U - 1) * P < hi; i += U * P) {
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
    for (; i < hi; i += P) {
        const float w = d[i] * v[i];
        v[i] = w;
        comp_add(acc, w * w);
    }
}

__device__ __forceinline__ void loop_normalise(float* __restrict__ v, int64_t lo, int64_t hi,
                                               float r) {
    constexpr int U = kGenericUnroll;
    const int64_t P = blockDim.x;
    int64_t i = lo + threadIdx.x;
    for (; i + (U - 1) * P < hi; i += U * P) {
        float b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) b[u] = v[i + u * P];
#pragma unroll
        for (int u = 0; u < U; ++u) v[i + u * P] = b[u] * r;
    }
    for (; i < hi; i += P) v[i] *= r;
}

// Poll one slot word for `tag`, bounded like poll_slot_word; every 256 polls
// it also looks at *status, so once one poll of the launch has timed out the
// others give up at once instead of each waiting out its own limit.
__device__ __forceinline__ uint32_t gather_word(const uint64_t* w, uint32_t tag, uint32_t* status) {
    for (uint32_t polls = 1;; ++polls) {
        const uint64_t x = load_slot_word(w);
        if ((uint32_t)(x >> 32) == tag) return (uint32_t)x;
        if (polls >= kPollLimit) {
            __hip_atomic_fetch_or(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return (uint32_t)x;
        }
        if ((polls & 255) == 0 &&
            (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u))
            return (uint32_t)x;
        __builtin_amdgcn_s_sleep(1);
    }
}

// All-gather: every team's partial of this step, combined in team order
// (thread t takes teams t, t + P, ...; then the team tree).  Result valid in
// thread 0.
__device__ __forceinline__ ff_t gather_partials(const uint64_t* set, int64_t T, uint32_t tag,
                                                uint32_t* status, ff_t* lds) {
    using R = Red<DT_F32, OP_SUM>;
    ff_t c = R::identity();
    for (int64_t i = threadIdx.x; i < T; i += blockDim.x) {
        const uint64_t* slot = set + i * kSlotWords;
        ff_t p;
        p.hi = __uint_as_float(gather_word(slot, tag, status));
        p.lo = __uint_as_float(gather_word(slot + 1, tag, status));
        c = R::combine(c, p);
    }
    __syncthreads();   // lds may still be read by the previous tree
    return team_reduce<R>(c, lds);
}

template <bool TEAMS>
__global__ __launch_bounds__(1024) void generic_power_kernel(const float* __restrict__ d,
                                                             float* __restrict__ v, int64_t n,
                                                             int iters, float* __restrict__ lambda,
                                                             CrossTeam ct) {
    using R = Red<DT_F32, OP_SUM>;
    __shared__ int s_work;       // the work descriptor: which loop runs next
    __shared__ float s_scale;    // and its argument
    __shared__ ff_t s_red[kMaxWaves];
    __shared__ ff_t s_sum;       // result of the last reduction loop
    const int tid = threadIdx.x;
    const int64_t T = gridDim.x;
    const Range blk = TEAMS ? bal_share(n, T, blockIdx.x) : Range{0, n};
    const uint32_t epoch = TEAMS ? read_epoch(ct.epoch) : 0u;
    int k = 0;   // steps completed (every thread follows the descriptors)
    // the main thread's sequential state (only thread 0's copy is used)
    int last = WORK_EXIT;
    float s = 0.0f;
    for (;;) {
        if (tid == 0) {   // sequential code
            if (last == WORK_SCALE_SQUARES) {
                s = s_sum.hi + s_sum.lo;
                s_scale = 1.0f / sqrtf(s);
                s_work = WORK_NORMALISE;
            } else if (k == iters) {
                if (blockIdx.x == 0) lambda[0] = sqrtf(s);
                s_work = WORK_EXIT;
            } else {
                s_work = WORK_SCALE_SQUARES;
            }
        }
        __syncthreads();   // the team picks up the work descriptor
        const int work = s_work;
        if (work == WORK_EXIT) break;
        if (work == WORK_SCALE_SQUARES) {
            ff_t acc = R::identity();
            loop_scale_squares(d, v, blk.lo, blk.hi, acc);
            acc = team_reduce<R>(acc, s_red);
            if constexpr (TEAMS) {
                const uint32_t tag = launch_tag(epoch + (uint32_t)k);
                uint64_t* set = ct.slots + (size_t)(k & 1) * T * kSlotWords;
                if (tid == 0) publish_tagged(acc, set + (size_t)blockIdx.x * kSlotWords, tag);
                acc = gather_partials(set, T, tag, ct.status, s_red);
            }
            if (tid == 0) s_sum = acc;
        } else {
            loop_normalise(v, blk.lo, blk.hi, s_scale);
            ++k;
        }
        __syncthreads();   // join: the loop is complete and its writes visible
        last = work;
    }
    // Every team read the epoch before publishing its first partial, and team
    // 0 has read every team's last partial: the next launch may take new tags.
    if (TEAMS && blockIdx.x == 0 && tid == 0)
        __hip_atomic_store(ct.epoch, epoch + (uint32_t)iters, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Teams of `threads` that can be resident at once on the current device.
static omprt_status coresident_teams(int threads, int* out) {
    int dev = 0;
    OMPRT_HIP(hipGetDevice(&dev));
    int coop = 0;
    OMPRT_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return fail(OMPRT_ERR_UNSUPPORTED, "device %d has no cooperative launch", dev);
    int per_cu = 0;
    OMPRT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(&generic_power_kernel<true>), threads, 0));
    *out = per_cu * device_cus();
    return OMPRT_OK;
}

}  // namespace omprt

using namespace omprt;

extern "C" omprt_status omprt_generic_power(const float* d_diag, float* d_v, int64_t n,
                                            int32_t iters, int32_t teams, int32_t threads,
                                            float* d_lambda, void* hip_stream) {
    if (n < 1 || n > ((int64_t)1 << 32))
        return fail(OMPRT_ERR_INVALID, "n = %lld outside 1..2^32", (long long)n);
    if (iters < 1) return fail(OMPRT_ERR_INVALID, "iters %d < 1", iters);
    if (teams < 0) return fail(OMPRT_ERR_INVALID, "teams %d < 0", teams);
    // default shape (measured at 2^10..2^20 elements, 100 steps): one team of
    // 512 threads while the loops are short, else teams of 256 threads, one
    // per 2048 elements, up to one per CU
    const bool auto_threads = threads == 0;
    if (auto_threads) threads = (teams == 1 || (teams == 0 && n <= 8192)) ? 512 : 256;
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
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int64_t want = teams != 0  ? teams
                         : auto_threads ? (n <= 8192 ? 1 : n / 2048)
                                        : n / ((int64_t)threads * 8);
    if (want <= 1) {
        teams = 1;
    } else {
        int maxco = 0;
        if (omprt_status st = coresident_teams(threads, &maxco)) return st;
        const int limit = std::min(maxco, kMaxGenericTeams);
        if (teams == 0)
            teams = (int)std::max<int64_t>(1, std::min<int64_t>(want, std::min(limit, device_cus())));
        else if (teams > limit)
            return fail(OMPRT_ERR_INVALID, "teams %d: at most %d teams of %d threads can be resident "
                        "at once here", teams, limit, threads);
    }
    hipError_t e;
    if (teams == 1) {
        hipLaunchKernelGGL(generic_power_kernel<false>, dim3(1), dim3(threads), 0, stream, d_diag,
                           d_v, n, (int)iters, d_lambda, CrossTeam{});
        e = hipGetLastError();
    } else {
        Workspace* ws = nullptr;
        if (omprt_status st = workspace_get(stream, 2 * teams, &ws)) return st;
        const CrossTeamArgs ca = ws->cross();
        CrossTeam ct{static_cast<uint64_t*>(ca.slots), ca.counter, ca.epoch, ca.status};
        int it = iters;
        void* args[] = {&d_diag, &d_v, &n, &it, &d_lambda, &ct};
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&generic_power_kernel<true>),
                                       dim3(teams), dim3(threads), args, 0, stream);
    }
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "generic launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}
