// stream.h -- the streaming part of a team's reduction: one team folds the
// element range [a, b) of an input into its lanes' private accumulators.
// Lanes read interleaved VB-byte vectors with nontemporal loads (one wave
// covers 64 * VB contiguous bytes per load), U loads in flight per lane; an
// element-wise head reaches VB alignment and an element-wise tail finishes.
#pragma once
#include "device.h"

namespace omprt {

// One VB-byte load of elements of type DT: T is a vector of the element type
// itself (loading a vector of dwords and rebuilding 64-bit elements from them
// lets the compiler split the load), bfloat16 excepted: its halves come out
// of dwords by shifts.
template <class S, int N>
struct VecType {
    using T = S __attribute__((ext_vector_type(N)));
    static __device__ __forceinline__ S get(const T& v, int k) { return v[k]; }
};
template <class S>
struct VecType<S, 1> {
    using T = S;
    static __device__ __forceinline__ S get(const T& v, int) { return v; }
};

template <int DT, int VB>
struct VecLoad {
    using S = typename DType<DT>::S;
    static constexpr int PER = VB / (int)sizeof(S);   // elements per load
    using VT = VecType<S, PER>;
    using T = typename VT::T;
    static __device__ __forceinline__ T load(const T* p) { return __builtin_nontemporal_load(p); }
    static __device__ __forceinline__ typename DType<DT>::V get(const T& v, int k) {
        return DType<DT>::from(VT::get(v, k));
    }
};
template <int VB>
struct VecLoad<DT_BF16, VB> {
    static constexpr int PER = VB / 2;
    using T = uint32_t __attribute__((ext_vector_type(VB / 4)));
    static __device__ __forceinline__ T load(const T* p) { return __builtin_nontemporal_load(p); }
    static __device__ __forceinline__ float get(const T& v, int k) {
        const uint32_t d = v[k >> 1];
        return __uint_as_float((k & 1) ? (d & 0xFFFF0000u) : (d << 16));
    }
};

template <class R, int DT, int VB>
__device__ __forceinline__ void accumulate_vec(typename R::Acc* acc,
                                               const typename VecLoad<DT, VB>::T& v) {
    using L = VecLoad<DT, VB>;
#pragma unroll
    for (int e = 0; e < L::PER; ++e) R::elem(acc[e % R::kNA], L::get(v, e));
}

// Streaming with any accumulation policy R (elem, kNA, Acc); acc has
// R::kNA entries; every thread of the team calls this with the same [a, b).
template <class R, int DT, int VB, int U>
__device__ __forceinline__ void stream_range_with(const typename DType<DT>::S* __restrict__ in,
                                                  int64_t a, int64_t b, typename R::Acc* acc) {
    using D = DType<DT>;
    using S = typename D::S;
    using L = VecLoad<DT, VB>;
    using Vec = typename L::T;
    constexpr int PER = L::PER;   // elements per vector
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
        for (int u = 0; u < U; ++u) r[u] = L::load(vp + v + (int64_t)u * P);
#pragma unroll
        for (int u = 0; u < U; ++u) accumulate_vec<R, DT, VB>(acc, r[u]);
    }
    for (; v < nv; v += P) {
        const Vec r = L::load(vp + v);
        accumulate_vec<R, DT, VB>(acc, r);
    }
    const int64_t t0 = p0 + nv * PER;
    if (tid < b - t0) R::elem(acc[0], D::from(in[t0 + tid]));
}

// The plain reduction's streaming: policy Red<DT, OP>.
template <int DT, int OP, int VB, int U>
__device__ __forceinline__ void stream_range(const typename DType<DT>::S* __restrict__ in,
                                             int64_t a, int64_t b,
                                             typename Red<DT, OP>::Acc* acc) {
    stream_range_with<Red<DT, OP>, DT, VB, U>(in, a, b, acc);
}

}  // namespace omprt
