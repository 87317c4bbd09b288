// reduce.hip -- the plain reduction kernel (one launch per reduction) and
// the empty-region kernel.
//
// reduce_kernel<DT, OP, VB, U>: team k = workgroup k reduces the balanced
// static distribute block bal(n, T, k) of the input (stream.h).  Per-lane
// partials are combined by the wave64 DPP reduction and the LDS tree, and
// teams combine through tagged cross-team slots and the wrap-increment
// last-team election (device.h).
#include "device.h"
#include "launch.h"
#include "stream.h"

namespace omprt {

template <int DT, int OP, int VB, int U>
__global__ __launch_bounds__(1024) void reduce_kernel(
    const typename DType<DT>::S* __restrict__ in, int64_t n,
    typename Red<DT, OP>::Out* __restrict__ x, CrossTeam ct) {
    using R = Red<DT, OP>;
    using Acc = typename R::Acc;

    __shared__ Acc lds_slots[kMaxWaves];
    __shared__ int s_last;

    const int64_t T = gridDim.x;
    const int tid = threadIdx.x;
    const uint32_t epoch = T > 1 ? read_epoch(ct.epoch) : 0u;
    const Range blk = bal_share(n, T, blockIdx.x);

    Acc acc[R::kNA];
#pragma unroll
    for (int i = 0; i < R::kNA; ++i) acc[i] = R::identity();

    stream_range<DT, OP, VB, U>(in, blk.lo, blk.hi, acc);

    Acc t = acc[0];
#pragma unroll
    for (int i = 1; i < R::kNA; ++i) t = R::combine(t, acc[i]);
    t = team_reduce<R>(t, lds_slots);

    if (T == 1) {   // single team: no cross-team step
        if (tid == 0) x[0] = R::finish(t, x[0]);
        return;
    }
    const uint32_t tag = launch_tag(epoch);
    if (!publish_and_elect(t, ct.slots + (size_t)blockIdx.x * kSlotWords, ct.counter,
                           (uint32_t)(T - 1), tag, &s_last))
        return;
    const Acc c = combine_slots<R>(ct.slots, T, tag, ct.status, lds_slots);
    if (tid == 0) {
        x[0] = R::finish(c, x[0]);
        advance_epoch(ct.epoch, epoch);
    }
}

static CrossTeam to_device_ct(const CrossTeamArgs& a) {
    return CrossTeam{static_cast<uint64_t*>(a.slots), a.counter, a.epoch, a.status};
}

// ---------------------------------------------------------------- dispatch

template <int DT, int OP, int VB, int U>
static hipError_t launch_one(const void* in, int64_t n, void* x, int teams, int threads,
                             const CrossTeamArgs& ct, hipStream_t stream) {
    using R = Red<DT, OP>;
    hipLaunchKernelGGL((reduce_kernel<DT, OP, VB, U>), dim3(teams), dim3(threads), 0, stream,
                       static_cast<const typename DType<DT>::S*>(in), n,
                       static_cast<typename R::Out*>(x), to_device_ct(ct));
    return hipGetLastError();
}

using Launcher = hipError_t (*)(const void*, int64_t, void*, int, int, const CrossTeamArgs&,
                                hipStream_t);

static int unroll_index(int u) { return u == 1 ? 0 : u == 2 ? 1 : u == 4 ? 2 : u == 8 ? 3 : -1; }
static int vec_index(int vb) { return vb == 8 ? 0 : vb == 16 ? 1 : -1; }

template <int DT, int OP, int VB>
struct UnrollRow {
    static constexpr Launcher row[4] = {launch_one<DT, OP, VB, 1>, launch_one<DT, OP, VB, 2>,
                                        launch_one<DT, OP, VB, 4>, launch_one<DT, OP, VB, 8>};
};

template <int DT, int OP>
static Launcher pick(int vi, int ui) {
    return vi == 0 ? UnrollRow<DT, OP, 8>::row[ui] : UnrollRow<DT, OP, 16>::row[ui];
}

template <int DT, int OP>
static Launcher pick_if(int vi, int ui) {
    if constexpr (op_defined(DT, OP))
        return pick<DT, OP>(vi, ui);
    else
        return nullptr;
}

template <int DT>
static Launcher pick_op(int op, int vi, int ui) {
    switch (op) {
        case OP_SUM: return pick_if<DT, OP_SUM>(vi, ui);
        case OP_MAX: return pick_if<DT, OP_MAX>(vi, ui);
        case OP_MIN: return pick_if<DT, OP_MIN>(vi, ui);
        case OP_PROD: return pick_if<DT, OP_PROD>(vi, ui);
        case OP_BAND: return pick_if<DT, OP_BAND>(vi, ui);
        case OP_BOR: return pick_if<DT, OP_BOR>(vi, ui);
        case OP_BXOR: return pick_if<DT, OP_BXOR>(vi, ui);
        case OP_LAND: return pick_if<DT, OP_LAND>(vi, ui);
        case OP_LOR: return pick_if<DT, OP_LOR>(vi, ui);
    }
    return nullptr;
}

static Launcher find_launcher(int dtype, int op, int vec_bytes, int unroll) {
    const int vi = vec_index(vec_bytes), ui = unroll_index(unroll);
    if (vi < 0 || ui < 0 || op < 0 || op >= OP_COUNT) return nullptr;
    switch (dtype) {
        case DT_I32: return pick_op<DT_I32>(op, vi, ui);
        case DT_I64: return pick_op<DT_I64>(op, vi, ui);
        case DT_F32: return pick_op<DT_F32>(op, vi, ui);
        case DT_F64: return pick_op<DT_F64>(op, vi, ui);
        case DT_BF16: return pick_op<DT_BF16>(op, vi, ui);
    }
    return nullptr;
}

bool reduce_variant_exists(int dtype, int op, int vec_bytes, int unroll) {
    return find_launcher(dtype, op, vec_bytes, unroll) != nullptr;
}

hipError_t launch_reduce(int dtype, int op, int vec_bytes, int unroll, const void* in,
                         int64_t n, void* x, int teams, int threads, const CrossTeamArgs& ct,
                         hipStream_t stream) {
    const Launcher f = find_launcher(dtype, op, vec_bytes, unroll);
    if (!f) return hipErrorInvalidValue;
    return f(in, n, x, teams, threads, ct, stream);
}

// ---------------------------------------------------------------- empty region

// A target region whose loop body does nothing but reduction(+: iters) with
// one count per iteration, so the launch carries the whole region protocol:
// every thread works out its static-schedule chunks (in closed form: the
// team's full distribute blocks share one per-thread count, only its last
// block can be partial) and checks its first and last chunk for consistency;
// the counts meet in the wave / LDS tree and the cross-team step, and the
// last team compares the total with n.  A thread with an inconsistent chunk,
// or a total other than n, sets status bit 16; iters (may be NULL) receives
// the total.
__global__ __launch_bounds__(1024) void empty_region_kernel(int64_t n, int P, int64_t dc,
                                                            int64_t c, int64_t* iters,
                                                            CrossTeam ct) {
    using R = Red<DT_I64, OP_SUM>;
    __shared__ uint64_t lds_slots[kMaxWaves];
    __shared__ int s_last;
    const int64_t T = gridDim.x, k = blockIdx.x;
    const int t = threadIdx.x;
    const uint32_t epoch = T > 1 ? read_epoch(ct.epoch) : 0u;
    uint64_t cnt = 0;
    bool bad = false;
    const int64_t nb = t < P ? team_nblocks(n, T, dc, k) : 0;
    if (nb > 0) {
        const Range first = team_block(n, T, dc, k, 0);
        const Range last = team_block(n, T, dc, k, nb - 1);
        const int64_t m0 = first.hi - first.lo, m1 = last.hi - last.lo;
        cnt = (uint64_t)(thread_niters(m0, P, c, t) * (nb - 1) + thread_niters(m1, P, c, t));
        const int64_t nc = thread_nchunks(m0, P, c, t);
        if (nc > 0) {
            const Range a = thread_chunk(first.lo, m0, P, c, t, 0);
            const Range z = thread_chunk(first.lo, m0, P, c, t, nc - 1);
            bad = !(first.lo <= a.lo && a.lo < a.hi && a.hi <= z.hi && z.lo < z.hi &&
                    z.hi <= first.hi && (nc == 1 || a.hi <= z.lo));
        }
        if (nb > 1 && !(first.hi <= last.lo && last.hi <= n)) bad = true;
    }
    if (bad) __hip_atomic_fetch_or(ct.status, 16u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t total = team_reduce<R>(cnt, lds_slots);
    if (T > 1) {
        const uint32_t tag = launch_tag(epoch);
        if (!publish_and_elect(total, ct.slots + (size_t)blockIdx.x * kSlotWords, ct.counter,
                               (uint32_t)(T - 1), tag, &s_last))
            return;
        total = combine_slots<R>(ct.slots, T, tag, ct.status, lds_slots);
    }
    if (t == 0) {
        if (total != (uint64_t)n)
            __hip_atomic_fetch_or(ct.status, 16u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (iters) iters[0] = R::finish(total, iters[0]);
        if (T > 1) advance_epoch(ct.epoch, epoch);
    }
}

hipError_t launch_empty_region(int64_t n, int teams, int threads, int64_t dist_chunk,
                               int64_t chunk, int64_t* iters, const CrossTeamArgs& ct,
                               hipStream_t stream) {
    const int block = (threads + kWave - 1) / kWave * kWave;
    hipLaunchKernelGGL(empty_region_kernel, dim3(teams), dim3(block), 0, stream, n, threads,
                       dist_chunk, chunk, iters, to_device_ct(ct));
    return hipGetLastError();
}

}  // namespace omprt
