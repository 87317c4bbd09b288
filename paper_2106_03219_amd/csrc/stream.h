// stream.h -- the streaming part of a team's reduction: one team folds the
// element range [a, b) of an input into its lanes' private accumulators.
// Lanes read interleaved VB-byte vectors with nontemporal loads (one wave
// covers 64 * VB contiguous bytes per load), U loads in flight per lane; an
// element-wise head reaches VB alignment and an element-wise tail finishes.
#pragma once
#include "device.h"

namespace omprt {

template <int VB>
struct VecOf;
template <>
struct VecOf<16> {
    using T = u32x4;
    static constexpr int kDwords = 4;
};
template <>
struct VecOf<8> {
    using T = u32x2;
    static constexpr int kDwords = 2;
};

template <int DT, int OP, int VB>
__device__ __forceinline__ void accumulate_vec(typename Red<DT, OP>::Acc* acc,
                                               const typename VecOf<VB>::T& v) {
    using D = DType<DT>;
    using R = Red<DT, OP>;
    constexpr int DW = VecOf<VB>::kDwords;
    constexpr int PER = D::kPerDword2 * DW / 2;
    uint32_t w[DW];
#pragma unroll
    for (int i = 0; i < DW; ++i) w[i] = v[i];
#pragma unroll
    for (int e = 0; e < PER; ++e) R::elem(acc[e % R::kNA], D::at(w, e));
}

// acc has Red<DT,OP>::kNA entries; every thread of the team calls this with
// the same [a, b).
template <int DT, int OP, int VB, int U>
__device__ __forceinline__ void stream_range(const typename DType<DT>::S* __restrict__ in,
                                             int64_t a, int64_t b,
                                             typename Red<DT, OP>::Acc* acc) {
    using D = DType<DT>;
    using R = Red<DT, OP>;
    using S = typename D::S;
    using Vec = typename VecOf<VB>::T;
    constexpr int PER = D::kPerDword2 * VecOf<VB>::kDwords / 2;   // elements per vector
    if (a >= b) return;
    const int tid = threadIdx.x;
    const int P = blockDim.x;
    const uintptr_t mis = reinterpret_cast<uintptr_t>(in + a) & (VB - 1);
    int64_t head = (int64_t)(((VB - mis) & (VB - 1)) / sizeof(S));
    if (head > b - a) head = b - a;
    if (tid < head) R::elem(acc[0], D::from(in[a + tid]));
    const int64_t p0 = a + head;
    const int64_t nv = (b - p0) / PER;
    const Vec* __restrict__ vp = reinterpret_cast<const Vec*>(in + p0);
    int64_t v = tid;
    for (; v + (int64_t)(U - 1) * P < nv; v += (int64_t)U * P) {
        Vec r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = __builtin_nontemporal_load(vp + v + (int64_t)u * P);
#pragma unroll
        for (int u = 0; u < U; ++u) accumulate_vec<DT, OP, VB>(acc, r[u]);
    }
    for (; v < nv; v += P) {
        const Vec r = __builtin_nontemporal_load(vp + v);
        accumulate_vec<DT, OP, VB>(acc, r);
    }
    const int64_t t0 = p0 + nv * PER;
    if (tid < b - t0) R::elem(acc[0], D::from(in[t0 + tid]));
}

}  // namespace omprt
