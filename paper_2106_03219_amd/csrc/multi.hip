// multi.hip -- several reduction variables of one region over the same
// input, e.g. reduction(+: s) reduction(max: hi) reduction(min: lo) on one
// loop: one pass over the data updates every variable's private copy, and
// the copies travel together through the wave / team tree and the tagged
// last-team combine (a partial larger than 16 bytes spans several slots).
#include "device.h"
#include "launch.h"
#include "runtime.h"
#include "stream.h"

namespace omprt {

// MASK bit 0: sum, bit 1: max, bit 2: min.
template <int DT, int MASK>
struct MultiRed {
    using SR = Red<DT, OP_SUM>;
    using XR = Red<DT, OP_MAX>;
    using NR = Red<DT, OP_MIN>;
    struct Acc {
        typename SR::Acc s;
        typename XR::Acc mx;
        typename NR::Acc mn;
    };
    static constexpr int kNA = 2;
    static __device__ __forceinline__ Acc identity() {
        return Acc{SR::identity(), XR::identity(), NR::identity()};
    }
    static __device__ __forceinline__ void elem(Acc& a, typename DType<DT>::V v) {
        if constexpr (MASK & 1) SR::elem(a.s, v);
        if constexpr (MASK & 2) XR::elem(a.mx, v);
        if constexpr (MASK & 4) NR::elem(a.mn, v);
    }
    static __device__ __forceinline__ Acc combine(Acc a, Acc b) {
        if constexpr (MASK & 1) a.s = SR::combine(a.s, b.s);
        if constexpr (MASK & 2) a.mx = XR::combine(a.mx, b.mx);
        if constexpr (MASK & 4) a.mn = NR::combine(a.mn, b.mn);
        return a;
    }
};

template <int DT, int MASK, int U>
__global__ __launch_bounds__(1024) void reduce_multi_kernel(
    const typename DType<DT>::S* __restrict__ in, int64_t n, typename Red<DT, OP_SUM>::Out* x_sum,
    typename Red<DT, OP_MAX>::Out* x_max, typename Red<DT, OP_MIN>::Out* x_min, CrossTeam ct) {
    using R = MultiRed<DT, MASK>;
    using Acc = typename R::Acc;
    __shared__ Acc lds_slots[kMaxWaves];
    __shared__ int s_last;
    const int64_t T = gridDim.x;
    const uint32_t epoch = T > 1 ? read_epoch(ct.epoch) : 0u;
    const Range blk = bal_share(n, T, blockIdx.x);
    Acc acc[R::kNA];
#pragma unroll
    for (int i = 0; i < R::kNA; ++i) acc[i] = R::identity();
    stream_range_with<R, DT, 16, U>(in, blk.lo, blk.hi, acc);
    Acc t = acc[0];
#pragma unroll
    for (int i = 1; i < R::kNA; ++i) t = R::combine(t, acc[i]);
    t = team_reduce<R>(t, lds_slots);
    Acc c = t;
    if (T > 1) {
        const uint32_t tag = launch_tag(epoch);
        if (!publish_and_elect(t, ct.slots + (size_t)blockIdx.x * slot_words<Acc>(), ct.counter,
                               (uint32_t)(T - 1), tag, &s_last))
            return;
        c = combine_slots<R>(ct.slots, T, tag, ct.status, lds_slots);
    }
    if (threadIdx.x == 0) {
        if constexpr (MASK & 1) x_sum[0] = R::SR::finish(c.s, x_sum[0]);
        if constexpr (MASK & 2) x_max[0] = R::XR::finish(c.mx, x_max[0]);
        if constexpr (MASK & 4) x_min[0] = R::NR::finish(c.mn, x_min[0]);
        if (T > 1) advance_epoch(ct.epoch, epoch);
    }
}

// Slots (of kSlotWords words) one team's partial takes.
template <int DT>
static int multi_slots() {
    return slot_words<typename MultiRed<DT, 7>::Acc>() / kSlotWords;
}

using MultiLauncher = void (*)(const void*, int64_t, void* const*, int, int, const CrossTeam&,
                               hipStream_t);

template <int DT, int MASK, int U>
static void launch_multi(const void* in, int64_t n, void* const* x, int teams, int threads,
                         const CrossTeam& ct, hipStream_t stream) {
    hipLaunchKernelGGL((reduce_multi_kernel<DT, MASK, U>), dim3(teams), dim3(threads), 0, stream,
                       static_cast<const typename DType<DT>::S*>(in), n,
                       static_cast<typename Red<DT, OP_SUM>::Out*>(x[0]),
                       static_cast<typename Red<DT, OP_MAX>::Out*>(x[1]),
                       static_cast<typename Red<DT, OP_MIN>::Out*>(x[2]), ct);
}

template <int DT, int MASK>
static MultiLauncher multi_pick_u(int u) {
    return u == 2 ? launch_multi<DT, MASK, 2> : u == 4 ? launch_multi<DT, MASK, 4> : nullptr;
}
template <int DT>
static MultiLauncher multi_pick(int mask, int u) {
    switch (mask) {
        case 1: return multi_pick_u<DT, 1>(u);
        case 2: return multi_pick_u<DT, 2>(u);
        case 3: return multi_pick_u<DT, 3>(u);
        case 4: return multi_pick_u<DT, 4>(u);
        case 5: return multi_pick_u<DT, 5>(u);
        case 6: return multi_pick_u<DT, 6>(u);
        case 7: return multi_pick_u<DT, 7>(u);
    }
    return nullptr;
}
static MultiLauncher multi_launcher(int dtype, int mask, int u, int* slots) {
    switch (dtype) {
        case DT_I32: *slots = multi_slots<DT_I32>(); return multi_pick<DT_I32>(mask, u);
        case DT_I64: *slots = multi_slots<DT_I64>(); return multi_pick<DT_I64>(mask, u);
        case DT_F32: *slots = multi_slots<DT_F32>(); return multi_pick<DT_F32>(mask, u);
        case DT_F64: *slots = multi_slots<DT_F64>(); return multi_pick<DT_F64>(mask, u);
        case DT_BF16: *slots = multi_slots<DT_BF16>(); return multi_pick<DT_BF16>(mask, u);
    }
    return nullptr;
}

}  // namespace omprt

using namespace omprt;

extern "C" omprt_status omprt_reduce_multi(const void* d_in, int64_t n, int32_t dtype,
                                           int32_t nvars, const int32_t* h_ops,
                                           void* const* h_x, const omprt_config* cfg,
                                           void* hip_stream) {
    if (dtype < 0 || dtype >= DT_COUNT_ABI) return fail(OMPRT_ERR_UNSUPPORTED, "dtype %d", dtype);
    if (nvars < 1 || nvars > 3) return fail(OMPRT_ERR_INVALID, "nvars %d outside 1..3", nvars);
    if (!h_ops || !h_x) return fail(OMPRT_ERR_INVALID, "ops / x array is NULL");
    if (n < 0 || n > ((int64_t)1 << 50))
        return fail(OMPRT_ERR_INVALID, "n = %lld outside 0..2^50", (long long)n);
    if (n > 0 && !d_in) return fail(OMPRT_ERR_INVALID, "input is NULL with n > 0");
    if (reinterpret_cast<uintptr_t>(d_in) % dtype_bytes(dtype))
        return fail(OMPRT_ERR_INVALID, "input is not aligned to its element size");
    void* x[3] = {nullptr, nullptr, nullptr};
    int mask = 0;
    for (int v = 0; v < nvars; ++v) {
        const int op = h_ops[v];
        if (op != OP_SUM && op != OP_MAX && op != OP_MIN)
            return fail(OMPRT_ERR_UNSUPPORTED, "variable %d: op %d (SUM, MAX or MIN)", v, op);
        if (mask & (1 << op)) return fail(OMPRT_ERR_INVALID, "op %d given twice", op);
        if (!h_x[v]) return fail(OMPRT_ERR_INVALID, "variable %d: x is NULL", v);
        if (reinterpret_cast<uintptr_t>(h_x[v]) % out_bytes(dtype, op))
            return fail(OMPRT_ERR_INVALID, "variable %d: x misaligned", v);
        mask |= 1 << op;
        x[op] = h_x[v];
    }
    if (cfg && cfg->vec_bytes && cfg->vec_bytes != 16)
        return fail(OMPRT_ERR_INVALID, "vec_bytes %d: this kernel loads 16 bytes", cfg->vec_bytes);
    if (cfg && cfg->unroll && cfg->unroll != 2 && cfg->unroll != 4)
        return fail(OMPRT_ERR_INVALID, "unroll %d: 2 or 4", cfg->unroll);
    omprt_config c2 = cfg ? *cfg : omprt_config{};
    c2.vec_bytes = 16;
    c2.flags |= OMPRT_CFG_NO_MODEL;
    LaunchCfg lc;
    if (omprt_status st = resolve_config(n, dtype, OP_SUM, 0, -1, &c2, &lc, nullptr)) return st;
    if (lc.unroll != 2 && lc.unroll != 4) lc.unroll = 4;
    if (n == 0) return OMPRT_OK;
    int slots = 1;
    const MultiLauncher f = multi_launcher(dtype, mask, lc.unroll, &slots);
    if (!f) return fail(OMPRT_ERR_UNSUPPORTED, "no fused kernel for this combination");
    if ((int64_t)lc.teams * slots > 65535 * 4)
        return fail(OMPRT_ERR_INVALID, "num_teams %d too large for the fused partials", lc.teams);
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    Workspace* ws = nullptr;
    if (omprt_status st = workspace_get(stream, lc.teams * slots, &ws)) return st;
    const CrossTeamArgs ca = ws->cross();
    const CrossTeam ct{static_cast<uint64_t*>(ca.slots), ca.counter, ca.epoch, ca.status};
    f(d_in, n, x, lc.teams, lc.threads, ct, stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "multi launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}
