// exact.hip -- the plain reduction under the exact static schedule, for
// comparison: team k reduces the static distribute block bal(n, T, k) (as
// the plain kernel does) and thread t of the team reduces exactly the
// iterations schedule(static) gives it, the contiguous run bal(m, P, t) of
// the block, in increasing order.  The plain kernel instead lets a team's
// lanes read interleaved 16-byte vectors -- allowed because a reduction
// body cannot tell which thread ran an iteration -- and that is what keeps
// its loads coalesced.  Here neighbouring lanes' runs lie m/P elements
// apart; for teams of whole waves the runs' whole lines pass through LDS
// (lines.h) so that every load instruction still covers whole lines, and
// each lane folds its own lines.  Otherwise, and for the ragged ends of the
// runs, each lane loads its own run (16-byte vectors, four in flight).
// Integer, max and min results equal the plain kernel's; sums may differ
// only by rounding order.
#include "device.h"
#include "launch.h"
#include "lines.h"
#include "runtime.h"
#include "stream.h"

namespace omprt {

// LINES: runs go through LDS a line at a time (8 KiB of dynamic LDS a wave;
// the host enables it for teams of whole waves).
template <int DT, int OP, bool LINES>
__global__ __launch_bounds__(1024) void reduce_exact_kernel(
    const typename DType<DT>::S* __restrict__ in, int64_t n,
    typename Red<DT, OP>::Out* __restrict__ x, CrossTeam ct) {
    using R = Red<DT, OP>;
    using Acc = typename R::Acc;
    using D = DType<DT>;
    using L = VecLoad<DT, 16>;
    using Vec = typename L::T;
    constexpr int PER = L::PER;
    constexpr int U = 4;
    extern __shared__ u32x4 stage_words[];
    __shared__ Acc lds_slots[kMaxWaves];
    __shared__ int s_last;
    const int64_t T = gridDim.x;
    const int tid = threadIdx.x;
    const uint32_t epoch = T > 1 ? read_epoch(ct.epoch) : 0u;
    const Range blk = bal_share(n, T, blockIdx.x);
    const Range own = bal_share(blk.hi - blk.lo, blockDim.x, tid);
    int64_t lo = blk.lo + own.lo;
    const int64_t hi = blk.lo + own.hi;

    Acc acc[R::kNA];
#pragma unroll
    for (int i = 0; i < R::kNA; ++i) acc[i] = R::identity();
    if (LINES) {
        // the part before the next line boundary by the lane alone, then as
        // many whole lines as every lane of the wave has, through LDS; the
        // rest below, by the lane alone
        constexpr int S = (int)sizeof(typename D::S);
        int64_t l0, np;
        run_lines<S>(in, lo, hi, l0, np);
        for (int64_t i = lo; i < l0; ++i) R::elem(acc[0], D::from(in[i]));
        line_fold<R, DT>(in, l0, np, stage_words + (size_t)(tid / kWave) * kStageSlots, acc);
        lo = l0 + np * (kLineBytes / S);
    }
    if (lo < hi) {
        const uintptr_t mis = reinterpret_cast<uintptr_t>(in + lo) & 15;
        int64_t head = (int64_t)(((16 - mis) & 15) / sizeof(typename D::S));
        if (head > hi - lo) head = hi - lo;
        for (int64_t i = lo; i < lo + head; ++i) R::elem(acc[0], D::from(in[i]));
        const int64_t p0 = lo + head;
        const int64_t nv = (hi - p0) / PER;
        const Vec* __restrict__ vp = reinterpret_cast<const Vec*>(in + p0);
        int64_t v = 0;
        for (; v + U <= nv; v += U) {
            Vec r[U];
#pragma unroll
            for (int u = 0; u < U; ++u) r[u] = L::load(vp + v + u);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < PER; ++e) R::elem(acc[e % R::kNA], L::get(r[u], e));
        }
        for (; v < nv; ++v) {
            const Vec r = L::load(vp + v);
#pragma unroll
            for (int e = 0; e < PER; ++e) R::elem(acc[e % R::kNA], L::get(r, e));
        }
        for (int64_t i = p0 + nv * PER; i < hi; ++i) R::elem(acc[0], D::from(in[i]));
    }
    Acc t = acc[0];
#pragma unroll
    for (int i = 1; i < R::kNA; ++i) t = R::combine(t, acc[i]);
    t = team_reduce<R>(t, lds_slots);
    if (T == 1) {
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

template <int DT, int OP>
static hipError_t launch_exact_one(const void* in, int64_t n, void* x, int teams, int threads,
                                   const CrossTeamArgs& a, hipStream_t stream) {
    const CrossTeam ct{static_cast<uint64_t*>(a.slots), a.counter, a.epoch, a.status};
    const auto* src = static_cast<const typename DType<DT>::S*>(in);
    auto* dst = static_cast<typename Red<DT, OP>::Out*>(x);
    if (threads % kWave != 0) {
        hipLaunchKernelGGL((reduce_exact_kernel<DT, OP, false>), dim3(teams), dim3(threads), 0,
                           stream, src, n, dst, ct);
        return hipGetLastError();
    }
    const size_t lds = (size_t)(threads / kWave) * kStageSlots * 16;
    if (lds > 64 * 1024) {   // past the default dynamic LDS limit: ask for it
        const hipError_t attr = hipFuncSetAttribute(
            reinterpret_cast<const void*>(reduce_exact_kernel<DT, OP, true>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (attr != hipSuccess) return attr;
    }
    hipLaunchKernelGGL((reduce_exact_kernel<DT, OP, true>), dim3(teams), dim3(threads), lds,
                       stream, src, n, dst, ct);
    return hipGetLastError();
}

template <int DT>
static hipError_t launch_exact_dt(int op, const void* in, int64_t n, void* x, int teams,
                                  int threads, const CrossTeamArgs& ct, hipStream_t stream) {
    switch (op) {
        case OP_SUM: return launch_exact_one<DT, OP_SUM>(in, n, x, teams, threads, ct, stream);
        case OP_MAX: return launch_exact_one<DT, OP_MAX>(in, n, x, teams, threads, ct, stream);
        case OP_MIN: return launch_exact_one<DT, OP_MIN>(in, n, x, teams, threads, ct, stream);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_reduce_exact(int dtype, int op, const void* in, int64_t n, void* x, int teams,
                               int threads, const CrossTeamArgs& ct, hipStream_t stream) {
    switch (dtype) {
        case DT_I32: return launch_exact_dt<DT_I32>(op, in, n, x, teams, threads, ct, stream);
        case DT_I64: return launch_exact_dt<DT_I64>(op, in, n, x, teams, threads, ct, stream);
        case DT_F32: return launch_exact_dt<DT_F32>(op, in, n, x, teams, threads, ct, stream);
        case DT_F64: return launch_exact_dt<DT_F64>(op, in, n, x, teams, threads, ct, stream);
        case DT_BF16: return launch_exact_dt<DT_BF16>(op, in, n, x, teams, threads, ct, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace omprt
