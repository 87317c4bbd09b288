// loc.hip -- maxloc / minloc: the largest (smallest) value of an input with
// its position, the common user-defined reduction.  Pairs (value, position)
// are ordered by value, then by the smaller position, so any combination
// order gives the same pair; floating NaNs never win.  Teams reduce the
// balanced block bal(n, T, k) with the streaming loads of the plain kernel,
// and the pairs go through the same wave / team tree and tagged last-team
// combine as any other reduction variable.
#include "device.h"
#include "launch.h"
#include "runtime.h"
#include "stream.h"

namespace omprt {

template <class V>
struct LocPair {   // 16 bytes: a value of up to 8 bytes, then the position
    V v;
    uint32_t pad;
    int64_t i;
};
template <>
struct LocPair<double> {
    double v;
    int64_t i;
};
template <>
struct LocPair<int64_t> {
    int64_t v;
    int64_t i;
};

template <int DT, int OP>
struct LocRed {
    using V = typename DType<DT>::V;
    using Acc = LocPair<V>;
    static __device__ __forceinline__ V worst() {
        if constexpr (DT == DT_I32) return OP == OP_MAX ? (V)INT32_MIN : (V)INT32_MAX;
        else if constexpr (DT == DT_I64) return OP == OP_MAX ? (V)INT64_MIN : (V)INT64_MAX;
        else return OP == OP_MAX ? -(V)__builtin_huge_val() : (V)__builtin_huge_val();
    }
    static __device__ __forceinline__ Acc make(V v, int64_t i) {
        Acc a{};
        a.v = v;
        a.i = i;
        return a;
    }
    static __device__ __forceinline__ Acc identity() { return make(worst(), INT64_MAX); }
    // true when a comes before b in the order (better value, then smaller position)
    static __device__ __forceinline__ bool before(const Acc& a, const Acc& b) {
        if constexpr (DT != DT_I32 && DT != DT_I64) {
            if (a.v != a.v) return false;   // NaN never wins
            if (b.v != b.v) return true;
        }
        if (a.v != b.v) return OP == OP_MAX ? a.v > b.v : a.v < b.v;
        return a.i < b.i;
    }
    static __device__ __forceinline__ Acc combine(Acc a, Acc b) { return before(b, a) ? b : a; }
    static __device__ __forceinline__ void elem(Acc& a, V v, int64_t i) {
        // a lane meets its elements in increasing position: a tie keeps a.  A
        // NaN v fails the ordered compare, so it never wins, and a.v is never a
        // NaN (it starts at the identity and only takes values that won).
        if (OP == OP_MAX ? v > a.v : v < a.v) a = make(v, i);
    }
};

template <int DT, int OP, int U>
__global__ __launch_bounds__(1024) void reduce_loc_kernel(const typename DType<DT>::S* __restrict__ in,
                                                          int64_t n,
                                                          typename DType<DT>::S* __restrict__ xval,
                                                          int64_t* __restrict__ xidx,
                                                          CrossTeam ct) {
    using R = LocRed<DT, OP>;
    using Acc = typename R::Acc;
    using D = DType<DT>;
    using L = VecLoad<DT, 16>;
    using Vec = typename L::T;
    constexpr int PER = L::PER;
    __shared__ Acc lds_slots[kMaxWaves];
    __shared__ int s_last;

    const int64_t T = gridDim.x;
    const int tid = threadIdx.x;
    const int P = blockDim.x;
    const uint32_t epoch = T > 1 ? read_epoch(ct.epoch) : 0u;
    const Range blk = bal_share(n, T, blockIdx.x);
    // one pair per element slot of a vector: independent compare chains; every
    // slot still meets its elements in increasing position
    Acc acc[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) acc[e] = R::identity();
    if (blk.lo < blk.hi) {
        const int64_t a = blk.lo, b = blk.hi;
        const uintptr_t mis = reinterpret_cast<uintptr_t>(in + a) & 15;
        int64_t head = (int64_t)(((16 - mis) & 15) / sizeof(typename D::S));
        if (head > b - a) head = b - a;
        if (tid < head) R::elem(acc[0], D::from(in[a + tid]), a + tid);
        const int64_t p0 = a + head;
        const int64_t nv = (b - p0) / PER;
        const Vec* __restrict__ vp = reinterpret_cast<const Vec*>(in + p0);
        int64_t v = tid;
        for (; v + (int64_t)(U - 1) * P < nv; v += (int64_t)U * P) {
            Vec r[U];
#pragma unroll
            for (int u = 0; u < U; ++u) r[u] = L::load(vp + v + (int64_t)u * P);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i0 = p0 + (v + (int64_t)u * P) * PER;
#pragma unroll
                for (int e = 0; e < PER; ++e) R::elem(acc[e], L::get(r[u], e), i0 + e);
            }
        }
        for (; v < nv; v += P) {
            const Vec r = L::load(vp + v);
            const int64_t i0 = p0 + v * PER;
#pragma unroll
            for (int e = 0; e < PER; ++e) R::elem(acc[e], L::get(r, e), i0 + e);
        }
        const int64_t t0 = p0 + nv * PER;
        if (tid < b - t0) R::elem(acc[0], D::from(in[t0 + tid]), t0 + tid);
    }
    Acc t = acc[0];
#pragma unroll
    for (int e = 1; e < PER; ++e) t = R::combine(t, acc[e]);
    t = team_reduce<R>(t, lds_slots);
    Acc c = t;
    if (T > 1) {
        const uint32_t tag = launch_tag(epoch);
        if (!publish_and_elect(t, ct.slots + (size_t)blockIdx.x * kSlotWords, ct.counter,
                               (uint32_t)(T - 1), tag, &s_last))
            return;
        c = combine_slots<R>(ct.slots, T, tag, ct.status, lds_slots);
    }
    if (tid == 0) {
        const Acc r = R::combine(R::make(D::from(xval[0]), xidx[0]), c);
        if constexpr (DT == DT_BF16)
            xval[0] = (uint16_t)(__float_as_uint(r.v) >> 16);   // a widened bf16: exact
        else
            xval[0] = r.v;
        xidx[0] = r.i;
        if (T > 1) advance_epoch(ct.epoch, epoch);
    }
}

using LocLauncher = void (*)(const void*, int64_t, void*, int64_t*, int, int, const CrossTeam&,
                             hipStream_t);

template <int DT, int OP, int U>
static void launch_loc(const void* in, int64_t n, void* xval, int64_t* xidx, int teams,
                       int threads, const CrossTeam& ct, hipStream_t stream) {
    using S = typename DType<DT>::S;
    hipLaunchKernelGGL((reduce_loc_kernel<DT, OP, U>), dim3(teams), dim3(threads), 0, stream,
                       static_cast<const S*>(in), n, static_cast<S*>(xval), xidx, ct);
}

template <int DT, int OP>
static LocLauncher loc_pick_u(int u) {
    switch (u) {
        case 1: return launch_loc<DT, OP, 1>;
        case 2: return launch_loc<DT, OP, 2>;
        case 4: return launch_loc<DT, OP, 4>;
        case 8: return launch_loc<DT, OP, 8>;
    }
    return nullptr;
}
template <int DT>
static LocLauncher loc_pick(int op, int u) {
    return op == OP_MAX ? loc_pick_u<DT, OP_MAX>(u) : loc_pick_u<DT, OP_MIN>(u);
}
static LocLauncher loc_launcher(int dtype, int op, int u) {
    switch (dtype) {
        case DT_I32: return loc_pick<DT_I32>(op, u);
        case DT_I64: return loc_pick<DT_I64>(op, u);
        case DT_F32: return loc_pick<DT_F32>(op, u);
        case DT_F64: return loc_pick<DT_F64>(op, u);
        case DT_BF16: return loc_pick<DT_BF16>(op, u);
    }
    return nullptr;
}

}  // namespace omprt

using namespace omprt;

extern "C" omprt_status omprt_reduce_loc(const void* d_in, int64_t n, int32_t dtype, int32_t op,
                                         void* d_val, int64_t* d_idx, const omprt_config* cfg,
                                         void* hip_stream) {
    if (dtype < 0 || dtype >= DT_COUNT_ABI) return fail(OMPRT_ERR_UNSUPPORTED, "dtype %d", dtype);
    if (op != OP_MAX && op != OP_MIN)
        return fail(OMPRT_ERR_UNSUPPORTED, "op %d (maxloc / minloc take MAX or MIN)", op);
    if (n < 0 || n > ((int64_t)1 << 50))
        return fail(OMPRT_ERR_INVALID, "n = %lld outside 0..2^50", (long long)n);
    if (!d_val || !d_idx) return fail(OMPRT_ERR_INVALID, "value/position is NULL");
    if (n > 0 && !d_in) return fail(OMPRT_ERR_INVALID, "input is NULL with n > 0");
    const int es = dtype_bytes(dtype);
    if ((reinterpret_cast<uintptr_t>(d_in) | reinterpret_cast<uintptr_t>(d_val)) % es ||
        reinterpret_cast<uintptr_t>(d_idx) % 8)
        return fail(OMPRT_ERR_INVALID, "misaligned input, value or position");
    if (cfg && cfg->vec_bytes && cfg->vec_bytes != 16)
        return fail(OMPRT_ERR_INVALID, "vec_bytes %d: maxloc / minloc load 16 bytes", cfg->vec_bytes);
    LaunchCfg lc;
    omprt_config c2 = cfg ? *cfg : omprt_config{};
    c2.vec_bytes = 16;
    c2.flags |= OMPRT_CFG_NO_MODEL;
    if (omprt_status st = resolve_config(n, dtype, OP_MAX, 0, -1, &c2, &lc, nullptr)) return st;
    // a pair per element slot keeps more compare chains going: eight loads in
    // flight do better here than the plain reduction's default (fp32 at 2^28:
    // 6.6 TB/s with eight, 5.4 with four)
    if (!(cfg && cfg->unroll)) lc.unroll = 8;
    if (n == 0) return OMPRT_OK;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    Workspace* ws = nullptr;
    if (omprt_status st = workspace_get(stream, lc.teams, &ws)) return st;
    const LocLauncher f = loc_launcher(dtype, op, lc.unroll);
    if (!f) return fail(OMPRT_ERR_INVALID, "unroll %d", lc.unroll);
    const CrossTeamArgs ca = ws->cross();
    const CrossTeam ct{static_cast<uint64_t*>(ca.slots), ca.counter, ca.epoch, ca.status};
    f(d_in, n, d_val, d_idx, lc.teams, lc.threads, ct, stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "loc launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}
