// array_kernel.h -- the array-section reduction kernel (reduction(op:
// x[0:m]) over a row-major rows x m block) and its launchers, templated on
// element type, operator, load width and unroll.  array.hip holds the host
// side; the instantiations are spread over one translation unit per
// element type (array_<type>.hip) so that they compile in parallel.
#pragma once
#include "device.h"
#include "launch.h"
#include "stream.h"

namespace omprt {

struct ArrayGeom {
    int64_t rows, m;
    int64_t W;            // columns per tile
    int64_t R;            // rows per period
    int64_t np;           // whole periods (rows / R)
    int32_t col_tiles;    // tiles
    int32_t rt;           // row teams per tile
    int32_t gs;           // teams per election group
    int32_t ng;           // groups per tile
};

struct ArrayCross {
    uint64_t* slots1;     // [rt][m] team partials, sizeof(Acc)/4 words each
    uint64_t* slots2;     // [ng][m] group partials (ng > 1)
    uint32_t* counters;   // [col_tiles][ng] group counters, then [col_tiles] tile counters
    uint32_t* done;       // tiles finished, 0 between launches
    uint32_t* epoch;
    uint32_t* status;
};

// Fold `count` tagged partials spaced `stride` words apart, in order.  The
// loads of up to kBatch partials are issued together; a word without this
// launch's tag (not yet visible) is polled on its own.
template <class R>
__device__ __forceinline__ typename R::Acc fold_tagged(const uint64_t* first, int64_t stride,
                                                       int count, uint32_t tag,
                                                       uint32_t* status) {
    using Acc = typename R::Acc;
    constexpr int NW = sizeof(Acc) / 4;
    constexpr int kBatch = NW <= 2 ? 16 : 8;
    Acc a = R::identity();
    for (int q0 = 0; q0 < count; q0 += kBatch) {
        // unconditional loads (a batch past the end re-reads the last
        // partial) keep the batch one straight run of loads
        uint64_t w[kBatch][NW];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int q = q0 + b < count ? q0 + b : count - 1;
#pragma unroll
            for (int i = 0; i < NW; ++i) w[b][i] = load_slot_word(first + q * stride + i);
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            if (q0 + b >= count) break;
            uint32_t p[NW];
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                uint64_t v = w[b][i];
                if ((uint32_t)(v >> 32) != tag)
                    v = poll_slot_word(first + (q0 + b) * stride + i, tag, status);
                p[i] = (uint32_t)v;
            }
            Acc y;
            __builtin_memcpy(&y, p, sizeof(Acc));
            a = R::combine(a, y);
        }
    }
    return a;
}

// Every thread of the team calls this after its stores; thread 0 takes part
// in the election.  True in every thread of the last team.
__device__ __forceinline__ bool elect_last(uint32_t* counter, uint32_t e, int* s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const uint32_t old = __builtin_amdgcn_atomic_inc32(counter, e, __ATOMIC_RELAXED, "agent");
        *s_flag = (old == e) ? 1 : 0;
    }
    __syncthreads();
    return *s_flag != 0;
}

// Fold the rows of the LDS matrix [nrows][wc] pairwise into row 0
// (nrows -> ceil(nrows / 2) -> ... -> 1).  Team-wide; ends with a barrier.
template <class R>
__device__ __forceinline__ void fold_rows(typename R::Acc* lds, int64_t nrows, int64_t wc) {
    const int P = blockDim.x;
    for (int64_t h = nrows; h > 1;) {
        const int64_t half = (h + 1) / 2;
        const int64_t cnt = (h - half) * wc;
        for (int64_t i = threadIdx.x; i < cnt; i += P) lds[i] = R::combine(lds[i], lds[i + half * wc]);
        __syncthreads();
        h = half;
    }
}

// The last team of a group folds the group's `count` published rows of wc
// partials (row q at first + q * stride words, column j at + j * NW) into
// lds[0 .. wc).  With fewer columns than threads, tpc = P / wc threads share
// a column: thread (q0, j) folds rows q0, q0 + tpc, ... in order, and the
// tpc results are folded pairwise in LDS.  Team-wide; ends with a barrier.
// lds must hold max(P, wc) entries.
template <class R>
__device__ __forceinline__ void fold_group(const uint64_t* first, int64_t stride, int count,
                                           int64_t wc, uint32_t tag, uint32_t* status,
                                           typename R::Acc* lds) {
    constexpr int NW = sizeof(typename R::Acc) / 4;
    const int P = blockDim.x, t = threadIdx.x;
    if (wc * 2 > P) {
        for (int64_t j = t; j < wc; j += P)
            lds[j] = fold_tagged<R>(first + j * NW, stride, count, tag, status);
        __syncthreads();
        return;
    }
    const int tpc = (int)(P / wc) < count ? (int)(P / wc) : count;
    const int q0 = t / (int)wc, j = t % (int)wc;
    if (q0 < tpc)
        lds[(int64_t)q0 * wc + j] = fold_tagged<R>(first + q0 * stride + j * NW, stride * tpc,
                                                   (count - q0 + tpc - 1) / tpc, tag, status);
    __syncthreads();
    fold_rows<R>(lds, tpc, wc);
}

// Loads of the streaming loop: one 16-byte vector (stream.h) or one element.
template <int DT, bool VEC>
struct ArrayLoad {
    using L = VecLoad<DT, 16>;
    using S = typename DType<DT>::S;
    using T = typename L::T;
    static constexpr int E = L::PER;
    static __device__ __forceinline__ T load(const S* p) {
        return L::load(reinterpret_cast<const T*>(p));
    }
    template <class R>
    static __device__ __forceinline__ void fold(typename R::Acc* acc, const T& v) {
#pragma unroll
        for (int k = 0; k < E; ++k) R::elem(acc[k], L::get(v, k));
    }
};
template <int DT>
struct ArrayLoad<DT, false> {
    using S = typename DType<DT>::S;
    using T = S;
    static constexpr int E = 1;
    static __device__ __forceinline__ T load(const S* p) { return __builtin_nontemporal_load(p); }
    template <class R>
    static __device__ __forceinline__ void fold(typename R::Acc* acc, const T& v) {
        R::elem(acc[0], DType<DT>::from(v));
    }
};

template <int DT, int OP, bool VEC, int U>
__global__ __launch_bounds__(512) void array_reduce_kernel(
    const typename DType<DT>::S* __restrict__ in, typename Red<DT, OP>::Out* __restrict__ x,
    ArrayGeom g, ArrayCross ct) {
    using D = DType<DT>;
    using R = Red<DT, OP>;
    using Acc = typename R::Acc;
    using S = typename D::S;
    using Ld = ArrayLoad<DT, VEC>;
    constexpr int E = Ld::E;
    constexpr int NW = sizeof(Acc) / 4;

    extern __shared__ __align__(16) unsigned char lds_raw[];
    Acc* lds = reinterpret_cast<Acc*>(lds_raw);
    __shared__ int s_last;

    const int tid = threadIdx.x;
    const int P = blockDim.x;
    const int c = (int)(blockIdx.x % (unsigned)g.col_tiles);
    const int r = (int)(blockIdx.x / (unsigned)g.col_tiles);
    const int64_t c0 = (int64_t)c * g.W;
    const int64_t wc = g.m - c0 < g.W ? g.m - c0 : g.W;
    const int64_t span = g.R * wc;
    const bool cross = g.rt > 1;
    const uint32_t epoch = cross ? read_epoch(ct.epoch) : 0u;

    // Lane slot u covers flat offsets o .. o + E - 1 of every period; aoff is
    // its element offset from the period's first element.  A slot past the
    // period's span reads the period's first vector instead and its copy is
    // never used: the loads stay unconditional, one straight run per period.
    int64_t aoff[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t o = ((int64_t)u * P + tid) * E;
        aoff[u] = o < span ? (o / wc) * g.m + (o % wc) : 0;
    }
    Acc acc[U][E];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < E; ++k) acc[u][k] = R::identity();

    const S* __restrict__ base = in + c0;
    const Range pr = bal_share(g.np, g.rt, r);
    for (int64_t p = pr.lo; p < pr.hi; ++p) {
        const S* __restrict__ bp = base + p * g.R * g.m;
        typename Ld::T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = Ld::load(bp + aoff[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) Ld::template fold<R>(acc[u], v[u]);
    }
    if (r == g.rt - 1) {   // rows after the whole periods, element by element
        const int64_t tl = (g.rows - g.np * g.R) * wc;
        if (tl > 0) {
            const S* __restrict__ bp = base + g.np * g.R * g.m;
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int64_t o = ((int64_t)u * P + tid) * E + k;
                    if (o < tl) R::elem(acc[u][k], D::from(bp[(o / wc) * g.m + (o % wc)]));
                }
        }
    }

    // Private copies -> LDS as a [rows][wc] matrix, whose rows are then
    // folded pairwise.  When every slot of a period is live and one layer of
    // P * E offsets holds whole rows, a lane's U slots are copies of the same
    // list items: they fold in registers first and LDS holds P * E / wc rows.
    const int64_t layer = (int64_t)P * E;
    const bool fold_u = U > 1 && span == U * layer && layer % wc == 0;
    int64_t nrows = g.R;
    if (fold_u) {
#pragma unroll
        for (int u = 1; u < U; ++u)
#pragma unroll
            for (int k = 0; k < E; ++k) acc[0][k] = R::combine(acc[0][k], acc[u][k]);
#pragma unroll
        for (int k = 0; k < E; ++k) lds[(int64_t)tid * E + k] = acc[0][k];
        nrows = layer / wc;
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int64_t o = ((int64_t)u * P + tid) * E + k;
                if (o < span) lds[o] = acc[u][k];
            }
    }
    __syncthreads();
    fold_rows<R>(lds, nrows, wc);

    if (!cross) {
        for (int64_t j = tid; j < wc; j += P) x[c0 + j] = R::finish(lds[j], x[c0 + j]);
        return;
    }

    const uint32_t tag = launch_tag(epoch);
    for (int64_t j = tid; j < wc; j += P)
        publish_tagged(lds[j], ct.slots1 + ((int64_t)r * g.m + c0 + j) * NW, tag);
    const int grp = r / g.gs;
    const int first = grp * g.gs;
    const int gsz = g.rt - first < g.gs ? g.rt - first : g.gs;
    if (!elect_last(ct.counters + (int64_t)c * g.ng + grp, (uint32_t)(gsz - 1), &s_last)) return;

    const int64_t stride = g.m * NW;
    fold_group<R>(ct.slots1 + ((int64_t)first * g.m + c0) * NW, stride, gsz, wc, tag, ct.status,
                  lds);
    if (g.ng == 1) {
        for (int64_t j = tid; j < wc; j += P) x[c0 + j] = R::finish(lds[j], x[c0 + j]);
    } else {
        for (int64_t j = tid; j < wc; j += P)
            publish_tagged(lds[j], ct.slots2 + ((int64_t)grp * g.m + c0 + j) * NW, tag);
        if (!elect_last(ct.counters + (int64_t)g.col_tiles * g.ng + c, (uint32_t)(g.ng - 1),
                        &s_last))
            return;
        fold_group<R>(ct.slots2 + c0 * NW, stride, g.ng, wc, tag, ct.status, lds);
        for (int64_t j = tid; j < wc; j += P) x[c0 + j] = R::finish(lds[j], x[c0 + j]);
    }
    // the tile is done; the last tile advances the epoch (every team of the
    // launch read it before publishing)
    if (tid == 0) {
        const uint32_t e = (uint32_t)(g.col_tiles - 1);
        if (__builtin_amdgcn_atomic_inc32(ct.done, e, __ATOMIC_RELAXED, "agent") == e)
            advance_epoch(ct.epoch, epoch);
    }
}

// ---------------------------------------------------------------- dispatch

using ArrayLauncher = void (*)(const void*, void*, const ArrayGeom&, const ArrayCross&, int,
                               size_t, hipStream_t);

template <int DT, int OP, bool VEC, int U>
static void launch_array_one(const void* in, void* x, const ArrayGeom& g, const ArrayCross& ct,
                             int threads, size_t lds, hipStream_t stream) {
    const unsigned teams = (unsigned)((int64_t)g.col_tiles * g.rt);
    hipLaunchKernelGGL((array_reduce_kernel<DT, OP, VEC, U>), dim3(teams), dim3(threads), lds,
                       stream, static_cast<const typename DType<DT>::S*>(in),
                       static_cast<typename Red<DT, OP>::Out*>(x), g, ct);
}

// Element loads: unroll 1..8.  16-byte loads: unroll 1..4 (eight vectors of
// private copies per lane would crowd out the registers).
template <int DT, int OP>
static ArrayLauncher array_pick_v(bool vec, int u) {
    if constexpr (!op_defined(DT, OP)) {
        return nullptr;
    } else {
        switch (u) {
            case 1: return vec ? launch_array_one<DT, OP, true, 1> : launch_array_one<DT, OP, false, 1>;
            case 2: return vec ? launch_array_one<DT, OP, true, 2> : launch_array_one<DT, OP, false, 2>;
            case 4: return vec ? launch_array_one<DT, OP, true, 4> : launch_array_one<DT, OP, false, 4>;
            case 8: return vec ? nullptr : launch_array_one<DT, OP, false, 8>;
        }
        return nullptr;
    }
}

// The launcher of one element type (array_<type>.hip instantiates it).
template <int DT>
ArrayLauncher array_launcher_impl(int op, bool vec, int u) {
    switch (op) {
        case OP_SUM: return array_pick_v<DT, OP_SUM>(vec, u);
        case OP_MAX: return array_pick_v<DT, OP_MAX>(vec, u);
        case OP_MIN: return array_pick_v<DT, OP_MIN>(vec, u);
        case OP_PROD: return array_pick_v<DT, OP_PROD>(vec, u);
        case OP_BAND: return array_pick_v<DT, OP_BAND>(vec, u);
        case OP_BOR: return array_pick_v<DT, OP_BOR>(vec, u);
        case OP_BXOR: return array_pick_v<DT, OP_BXOR>(vec, u);
        case OP_LAND: return array_pick_v<DT, OP_LAND>(vec, u);
        case OP_LOR: return array_pick_v<DT, OP_LOR>(vec, u);
    }
    return nullptr;
}

ArrayLauncher array_launcher_i32(int op, bool vec, int u);
ArrayLauncher array_launcher_i64(int op, bool vec, int u);
ArrayLauncher array_launcher_f32(int op, bool vec, int u);
ArrayLauncher array_launcher_f64(int op, bool vec, int u);
ArrayLauncher array_launcher_bf16(int op, bool vec, int u);

}  // namespace omprt
