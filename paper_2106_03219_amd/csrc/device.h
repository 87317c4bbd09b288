// device.h -- gfx950 device primitives of the data-parallel core:
// wave64 cross-lane reduction (DPP + bpermute), the intra-team tree through
// LDS with the team barrier, the cross-team publish / wrap-increment /
// last-team protocol, compensated (float-float) arithmetic, and the
// element-type and reduction-operator policies the kernels are templated on.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ops.h"
#include "sched.h"

namespace omprt {


typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kWave = 64;
constexpr int kMaxWaves = 1024 / kWave;

// ---------------------------------------------------------------- cross-lane

// GFX9 DPP controls used by the wave reduction (all stay inside a row of 16
// lanes, so every source lane exists when the wave is full).
enum : int {
    kDppQuadXor1 = 0xB1,   // quad_perm [1,0,3,2]
    kDppQuadXor2 = 0x4E,   // quad_perm [2,3,0,1]
    kDppRowRor4 = 0x124,   // row_ror:4
    kDppRowRor8 = 0x128,   // row_ror:8
};

template <int CTRL, class T>
__device__ __forceinline__ T dpp_move(const T& x) {
    static_assert(sizeof(T) % 4 == 0, "DPP moves whole dwords");
    constexpr int W = sizeof(T) / 4;
    int w[W];
    __builtin_memcpy(w, &x, sizeof(T));
#pragma unroll
    for (int i = 0; i < W; ++i) w[i] = __builtin_amdgcn_update_dpp(w[i], w[i], CTRL, 0xF, 0xF, false);
    T y;
    __builtin_memcpy(&y, w, sizeof(T));
    return y;
}

template <class T>
__device__ __forceinline__ T shfl_xor_words(const T& x, int mask) {
    static_assert(sizeof(T) % 4 == 0, "shuffles move whole dwords");
    constexpr int W = sizeof(T) / 4;
    int w[W];
    __builtin_memcpy(w, &x, sizeof(T));
#pragma unroll
    for (int i = 0; i < W; ++i) w[i] = __shfl_xor(w[i], mask, kWave);
    T y;
    __builtin_memcpy(&y, w, sizeof(T));
    return y;
}

// 64 lane partials -> 1 (every lane ends with a full combination; lane 0's
// value is the one used).  Must be called with all 64 lanes active.
template <class R>
__device__ __forceinline__ typename R::Acc wave_reduce(typename R::Acc a) {
    a = R::combine(a, dpp_move<kDppQuadXor1>(a));
    a = R::combine(a, dpp_move<kDppQuadXor2>(a));
    a = R::combine(a, dpp_move<kDppRowRor4>(a));
    a = R::combine(a, dpp_move<kDppRowRor8>(a));
    a = R::combine(a, shfl_xor_words(a, 16));
    a = R::combine(a, shfl_xor_words(a, 32));
    return a;
}

// Intra-team tree: each wave reduces, lane 0 of wave w writes LDS slot w,
// team barrier, wave 0 reduces the slots.  Slots past the wave count are
// never read (LDS is not zero-initialised).  Result valid in thread 0.
// blockDim.x must be a multiple of 64.
template <class R>
__device__ __forceinline__ typename R::Acc team_reduce(typename R::Acc a,
                                                       typename R::Acc* slots) {
    a = wave_reduce<R>(a);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    if (lane == 0) slots[wave] = a;
    __syncthreads();
    if (wave == 0) {
        a = lane < nw ? slots[lane] : R::identity();
        a = wave_reduce<R>(a);
    }
    return a;
}

// ---------------------------------------------------------------- cross-team

// Cross-team state of one launch.  A participant (team, or tile of a batched
// segment) publishes its partial into its slot; the wrap-around increment
//   { v = *counter; *counter = v >= e ? 0 : v + 1 }   (e = participants - 1)
// elects the one that reads e as the last; it combines every slot and leaves
// the counter at 0 for the next launch or graph replay.
//
// Visibility without a per-team fence: every 64-bit slot word carries a
// 32-bit payload and the launch's 32-bit tag and is written and read as an
// agent-scope atomic (coherent across the XCDs' L2s).  The last participant
// polls each word until it holds this launch's tag, so it never needs the
// publishing stores to be ordered before the increments.  (An agent-scope
// release fence per team -- the device-wide fence behind the OpenMP flush --
// costs an L2 writeback on gfx950 and throttles the whole grid.)  The tag
// comes from an epoch word in device memory that every participant reads at
// start and the launch's finisher advances at the end, so graph replays get
// fresh tags too.  Polls are bounded; a timeout sets *status.
struct CrossTeam {
    uint64_t* slots;     // kSlotWords words per participant
    uint32_t* counter;   // election counter, 0 between launches
    uint32_t* epoch;     // launch epoch
    uint32_t* status;    // set to 1 if a poll timed out
};
constexpr int kSlotWords = 4;                 // 32-bit payload words per slot
// Slot words a participant's partial of type Acc takes (whole slots: a
// partial larger than 16 bytes spans several).
template <class Acc>
constexpr int slot_words() {
    return ((int)(sizeof(Acc) / 4) + kSlotWords - 1) / kSlotWords * kSlotWords;
}
constexpr uint32_t kPollLimit = 1u << 22;     // polls per slot word before giving up

__device__ __forceinline__ uint32_t read_epoch(const uint32_t* epoch) {
    return __hip_atomic_load(const_cast<uint32_t*>(epoch), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void advance_epoch(uint32_t* epoch, uint32_t e) {
    __hip_atomic_store(epoch, e + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Odd, so zero-filled slots never match.
__device__ __forceinline__ uint32_t launch_tag(uint32_t epoch) { return (epoch << 1) | 1u; }

template <class Acc>
__device__ __forceinline__ void publish_tagged(const Acc& v, uint64_t* slot, uint32_t tag) {
    static_assert(sizeof(Acc) % 4 == 0, "partials are whole 32-bit words");
    constexpr int W = sizeof(Acc) / 4;
    uint32_t w[W];
    __builtin_memcpy(w, &v, sizeof(Acc));
#pragma unroll
    for (int i = 0; i < W; ++i)
        __hip_atomic_store(slot + i, ((uint64_t)tag << 32) | w[i], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t load_slot_word(const uint64_t* w) {
    return __hip_atomic_load(const_cast<uint64_t*>(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Poll one slot word until it carries `tag` (bounded; a timeout sets bit 1
// of *status and returns whatever the word holds).
__device__ __forceinline__ uint64_t poll_slot_word(const uint64_t* w, uint32_t tag,
                                                   uint32_t* status) {
    uint32_t polls = 0;
    for (;;) {
        const uint64_t v = load_slot_word(w);
        if ((uint32_t)(v >> 32) == tag) return v;
        if (++polls >= kPollLimit) {
            __hip_atomic_fetch_or(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return v;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

template <class Acc>
__device__ __forceinline__ Acc collect_tagged(const uint64_t* slot, uint32_t tag,
                                              uint32_t* status) {
    constexpr int W = sizeof(Acc) / 4;
    uint32_t w[W];
#pragma unroll
    for (int i = 0; i < W; ++i) w[i] = (uint32_t)poll_slot_word(slot + i, tag, status);
    Acc a;
    __builtin_memcpy(&a, w, sizeof(Acc));
    return a;
}

// Thread 0 publishes the team's partial and takes part in the election.
// Returns the same bool in every thread of the team: true for the last.
template <class Acc>
__device__ __forceinline__ bool publish_and_elect(const Acc& partial, uint64_t* slot,
                                                  uint32_t* counter, uint32_t e, uint32_t tag,
                                                  int* s_flag) {
    if (threadIdx.x == 0) {
        publish_tagged(partial, slot, tag);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);   // keep the stores before the increment
        const uint32_t old = __builtin_amdgcn_atomic_inc32(counter, e, __ATOMIC_RELAXED, "agent");
        *s_flag = (old == e) ? 1 : 0;
    }
    __syncthreads();
    return *s_flag != 0;
}

// Last participant: combine the partials [0, count) in index order (thread
// t takes t, t + P, ...; then the team tree).  Partial i starts at word
// i * slot_words<Acc>().  Result valid in thread 0.
template <class R>
__device__ __forceinline__ typename R::Acc combine_slots(const uint64_t* slots, int64_t count,
                                                         uint32_t tag, uint32_t* status,
                                                         typename R::Acc* lds) {
    using Acc = typename R::Acc;
    Acc c = R::identity();
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x)
        c = R::combine(c, collect_tagged<Acc>(slots + i * slot_words<Acc>(), tag, status));
    __syncthreads();   // lds may still be read by the previous tree
    return team_reduce<R>(c, lds);
}

// ---------------------------------------------------------------- float-float

template <class F>
struct Pair {
    F hi, lo;   // represents hi + lo
};
using ff_t = Pair<float>;
using dd_t = Pair<double>;

// Knuth's TwoSum: s + err == a + b exactly.
template <class F>
__device__ __forceinline__ Pair<F> two_sum(F a, F b) {
    const F s = a + b;
    const F bb = s - a;
    const F err = (a - (s - bb)) + (b - bb);
    return Pair<F>{s, err};
}

// Dekker's Fast2Sum, valid when |a| >= |b| or a == 0.
template <class F>
__device__ __forceinline__ Pair<F> fast_two_sum(F a, F b) {
    const F s = a + b;
    const F err = b - (s - a);
    return Pair<F>{s, err};
}

// Accurate float-float addition: both the high and the low parts go
// through TwoSum, then two renormalisations (no cancellation assumption).
template <class F>
__device__ __forceinline__ Pair<F> pair_add(Pair<F> x, Pair<F> y) {
    Pair<F> s = two_sum(x.hi, y.hi);
    const Pair<F> t = two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

// Compensated accumulation of one value: TwoSum captures the rounding error
// of hi + x exactly whatever the magnitudes (a Kahan/Fast2Sum step would
// need |hi| >= |x|, which sums crossing zero violate); the errors gather in
// lo.  The pair represents hi + lo.
template <class F>
__device__ __forceinline__ void comp_add(Pair<F>& a, F x) {
    const F s = a.hi + x;
    const F bb = s - a.hi;
    const F err = (a.hi - (s - bb)) + (x - bb);
    a.hi = s;
    a.lo += err;
}

// ---------------------------------------------------------------- element types

template <int DT>
struct DType;

template <>
struct DType<DT_I32> {
    using S = int32_t;   // storage
    using V = int32_t;   // computation value
    static constexpr int kPerDword2 = 2;   // elements per 2 dwords
    static __device__ __forceinline__ V from(S s) { return s; }
    static __device__ __forceinline__ V at(const uint32_t* w, int i) { return (int32_t)w[i]; }
};
template <>
struct DType<DT_I64> {
    using S = int64_t;
    using V = int64_t;
    static constexpr int kPerDword2 = 1;
    static __device__ __forceinline__ V from(S s) { return s; }
    static __device__ __forceinline__ V at(const uint32_t* w, int i) {
        return (int64_t)(((uint64_t)w[2 * i + 1] << 32) | w[2 * i]);
    }
};
template <>
struct DType<DT_F32> {
    using S = float;
    using V = float;
    static constexpr int kPerDword2 = 2;
    static __device__ __forceinline__ V from(S s) { return s; }
    static __device__ __forceinline__ V at(const uint32_t* w, int i) { return __uint_as_float(w[i]); }
};
template <>
struct DType<DT_F64> {
    using S = double;
    using V = double;
    static constexpr int kPerDword2 = 1;
    static __device__ __forceinline__ V from(S s) { return s; }
    static __device__ __forceinline__ V at(const uint32_t* w, int i) {
        return __hiloint2double((int)w[2 * i + 1], (int)w[2 * i]);
    }
};
// bfloat16 is the high half of a binary32: widening is a shift.
template <>
struct DType<DT_BF16> {
    using S = uint16_t;
    using V = float;
    static constexpr int kPerDword2 = 4;
    static __device__ __forceinline__ V from(S s) { return __uint_as_float((uint32_t)s << 16); }
    static __device__ __forceinline__ V at(const uint32_t* w, int i) {
        const uint32_t d = w[i >> 1];
        return __uint_as_float((i & 1) ? (d & 0xFFFF0000u) : (d << 16));
    }
};

// ---------------------------------------------------------------- reduction ops

// Every policy provides: Acc (<= 16 bytes, the per-lane / per-team state),
// Out (type of x), identity(), elem(Acc&, V), combine(Acc, Acc),
// finish(Acc, Out x_orig) -> Out, and kNA (independent per-lane
// accumulators the streaming loop keeps, for instruction-level parallelism).
template <int DT, int OP>
struct Red;

// Integer sums: wrap modulo 2^w, computed unsigned.
template <>
struct Red<DT_I32, OP_SUM> {
    using Acc = uint32_t;
    using Out = int32_t;
    static constexpr int kNA = 1;
    static __device__ __forceinline__ Acc identity() { return 0u; }
    static __device__ __forceinline__ void elem(Acc& a, int32_t v) { a += (uint32_t)v; }
    static __device__ __forceinline__ Acc combine(Acc a, Acc b) { return a + b; }
    static __device__ __forceinline__ Out finish(Acc a, Out x) { return (int32_t)((uint32_t)x + a); }
};
template <>
struct Red<DT_I64, OP_SUM> {
    using Acc = uint64_t;
    using Out = int64_t;
    static constexpr int kNA = 1;
    static __device__ __forceinline__ Acc identity() { return 0ull; }
    static __device__ __forceinline__ void elem(Acc& a, int64_t v) { a += (uint64_t)v; }
    static __device__ __forceinline__ Acc combine(Acc a, Acc b) { return a + b; }
    static __device__ __forceinline__ Out finish(Acc a, Out x) { return (int64_t)((uint64_t)x + a); }
};

// Signed integer max / min.
template <class I, int OP>
struct IntExt {
    using Acc = I;
    using Out = I;
    static constexpr int kNA = 1;
    static __device__ __forceinline__ Acc identity() {
        if (OP == OP_MAX) return sizeof(I) == 4 ? (I)INT32_MIN : (I)INT64_MIN;
        return sizeof(I) == 4 ? (I)INT32_MAX : (I)INT64_MAX;
    }
    static __device__ __forceinline__ Acc combine(Acc a, Acc b) {
        return OP == OP_MAX ? (a > b ? a : b) : (a < b ? a : b);
    }
    static __device__ __forceinline__ void elem(Acc& a, I v) { a = combine(a, v); }
    static __device__ __forceinline__ Out finish(Acc a, Out x) { return combine(a, x); }
};
template <> struct Red<DT_I32, OP_MAX> : IntExt<int32_t, OP_MAX> {};
template <> struct Red<DT_I32, OP_MIN> : IntExt<int32_t, OP_MIN> {};
template <> struct Red<DT_I64, OP_MAX> : IntExt<int64_t, OP_MAX> {};
template <> struct Red<DT_I64, OP_MIN> : IntExt<int64_t, OP_MIN> {};

// Floating max / min: IEEE maxNum / minNum (NaN-dropping), identity -/+inf.
template <class F, int OP>
struct FpExt {
    using Acc = F;
    static constexpr int kNA = 1;
    static __device__ __forceinline__ Acc identity() {
        return OP == OP_MAX ? -__builtin_huge_valf() : __builtin_huge_valf();
    }
    static __device__ __forceinline__ Acc combine(Acc a, Acc b) {
        return OP == OP_MAX ? __builtin_fmax(a, b) : __builtin_fmin(a, b);
    }
    static __device__ __forceinline__ void elem(Acc& a, F v) { a = combine(a, v); }
};
template <int OP>
struct FpExt32 : FpExt<float, OP> {
    using Out = float;
    static __device__ __forceinline__ float combine(float a, float b) {
        return OP == OP_MAX ? __builtin_fmaxf(a, b) : __builtin_fminf(a, b);
    }
    static __device__ __forceinline__ void elem(float& a, float v) { a = combine(a, v); }
    static __device__ __forceinline__ Out finish(float a, Out x) { return combine(a, x); }
};
template <int OP>
struct FpExt64 : FpExt<double, OP> {
    using Out = double;
    static __device__ __forceinline__ double identity() {
        return OP == OP_MAX ? -__builtin_huge_val() : __builtin_huge_val();
    }
    static __device__ __forceinline__ Out finish(double a, Out x) {
        return FpExt<double, OP>::combine(a, x);
    }
};
template <> struct Red<DT_F32, OP_MAX> : FpExt32<OP_MAX> {};
template <> struct Red<DT_F32, OP_MIN> : FpExt32<OP_MIN> {};
template <> struct Red<DT_F64, OP_MAX> : FpExt64<OP_MAX> {};
template <> struct Red<DT_F64, OP_MIN> : FpExt64<OP_MIN> {};

// bf16 max / min: compared as widened fp32; the result is one of the inputs
// (or x), so narrowing back to bf16 is exact truncation.
template <int OP>
struct Bf16Ext : FpExt32<OP> {
    using Out = uint16_t;
    static __device__ __forceinline__ Out finish(float a, Out x) {
        const float r = FpExt32<OP>::combine(a, __uint_as_float((uint32_t)x << 16));
        return (uint16_t)(__float_as_uint(r) >> 16);
    }
};
template <> struct Red<DT_BF16, OP_MAX> : Bf16Ext<OP_MAX> {};
template <> struct Red<DT_BF16, OP_MIN> : Bf16Ext<OP_MIN> {};

// Compensated sums: per-lane TwoSum accumulation in the working precision,
// float-float (or double-double) combination through the wave / team /
// cross-team tree.
template <class F, int NA>
struct CompSum {
    using Acc = Pair<F>;
    static constexpr int kNA = NA;
    static __device__ __forceinline__ Acc identity() { return Acc{F(0), F(0)}; }
    static __device__ __forceinline__ void elem(Acc& a, F v) { comp_add(a, v); }
    static __device__ __forceinline__ Acc combine(Acc a, Acc b) { return pair_add(a, b); }
};
template <> struct Red<DT_F32, OP_SUM> : CompSum<float, 4> {
    using Out = float;
    static __device__ __forceinline__ Out finish(Acc a, Out x) {
        return pair_add(a, Acc{x, 0.0f}).hi;
    }
};
template <> struct Red<DT_BF16, OP_SUM> : CompSum<float, 4> {
    using Out = float;   // bf16 sums return the fp32 accumulator
    static __device__ __forceinline__ Out finish(Acc a, Out x) {
        return pair_add(a, Acc{x, 0.0f}).hi;
    }
};
template <> struct Red<DT_F64, OP_SUM> : CompSum<double, 2> {
    using Out = double;
    static __device__ __forceinline__ Out finish(Acc a, Out x) {
        return pair_add(a, Acc{x, 0.0}).hi;
    }
};

// ---------------------------------------------------------------- more identifiers

// Integer product: wraps modulo 2^w (computed unsigned).
template <class I, class U>
struct IntProd {
    using Acc = U;
    using Out = I;
    static constexpr int kNA = 1;
    static __device__ __forceinline__ Acc identity() { return (U)1; }
    static __device__ __forceinline__ void elem(Acc& a, I v) { a *= (U)v; }
    static __device__ __forceinline__ Acc combine(Acc a, Acc b) { return a * b; }
    static __device__ __forceinline__ Out finish(Acc a, Out x) { return (I)((U)x * a); }
};
template <> struct Red<DT_I32, OP_PROD> : IntProd<int32_t, uint32_t> {};
template <> struct Red<DT_I64, OP_PROD> : IntProd<int64_t, uint64_t> {};

// Bitwise and / or / xor on integers.
template <class I, class U, int OP>
struct IntBits {
    using Acc = U;
    using Out = I;
    static constexpr int kNA = 1;
    static __device__ __forceinline__ Acc identity() { return OP == OP_BAND ? ~(U)0 : (U)0; }
    static __device__ __forceinline__ Acc combine(Acc a, Acc b) {
        return OP == OP_BAND ? (a & b) : OP == OP_BOR ? (a | b) : (a ^ b);
    }
    static __device__ __forceinline__ void elem(Acc& a, I v) { a = combine(a, (U)v); }
    static __device__ __forceinline__ Out finish(Acc a, Out x) { return (I)combine((U)x, a); }
};
template <> struct Red<DT_I32, OP_BAND> : IntBits<int32_t, uint32_t, OP_BAND> {};
template <> struct Red<DT_I32, OP_BOR> : IntBits<int32_t, uint32_t, OP_BOR> {};
template <> struct Red<DT_I32, OP_BXOR> : IntBits<int32_t, uint32_t, OP_BXOR> {};
template <> struct Red<DT_I64, OP_BAND> : IntBits<int64_t, uint64_t, OP_BAND> {};
template <> struct Red<DT_I64, OP_BOR> : IntBits<int64_t, uint64_t, OP_BOR> {};
template <> struct Red<DT_I64, OP_BXOR> : IntBits<int64_t, uint64_t, OP_BXOR> {};

// Logical and / or: an operand is true when it is not zero (NaN is true);
// the result is 0 or 1 in x's type (bf16: the bits of 1.0 or of 0.0).
template <class V, class O, int OP>
struct Logic {
    using Acc = uint32_t;
    using Out = O;
    static constexpr int kNA = 1;
    static __device__ __forceinline__ Acc identity() { return OP == OP_LAND ? 1u : 0u; }
    static __device__ __forceinline__ Acc combine(Acc a, Acc b) {
        return OP == OP_LAND ? (a & b) : (a | b);
    }
    static __device__ __forceinline__ void elem(Acc& a, V v) { a = combine(a, v != V(0) ? 1u : 0u); }
};
template <class I, int OP>
struct IntLogic : Logic<I, I, OP> {
    static __device__ __forceinline__ I finish(uint32_t a, I x) {
        return (I)Logic<I, I, OP>::combine(x != 0 ? 1u : 0u, a);
    }
};
template <class F, int OP>
struct FpLogic : Logic<F, F, OP> {
    static __device__ __forceinline__ F finish(uint32_t a, F x) {
        return Logic<F, F, OP>::combine(x != F(0) ? 1u : 0u, a) ? F(1) : F(0);
    }
};
template <int OP>
struct Bf16Logic : Logic<float, uint16_t, OP> {
    static __device__ __forceinline__ uint16_t finish(uint32_t a, uint16_t x) {
        const bool xt = __uint_as_float((uint32_t)x << 16) != 0.0f;
        return Logic<float, uint16_t, OP>::combine(xt ? 1u : 0u, a) ? (uint16_t)0x3F80 : (uint16_t)0;
    }
};
template <> struct Red<DT_I32, OP_LAND> : IntLogic<int32_t, OP_LAND> {};
template <> struct Red<DT_I32, OP_LOR> : IntLogic<int32_t, OP_LOR> {};
template <> struct Red<DT_I64, OP_LAND> : IntLogic<int64_t, OP_LAND> {};
template <> struct Red<DT_I64, OP_LOR> : IntLogic<int64_t, OP_LOR> {};
template <> struct Red<DT_F32, OP_LAND> : FpLogic<float, OP_LAND> {};
template <> struct Red<DT_F32, OP_LOR> : FpLogic<float, OP_LOR> {};
template <> struct Red<DT_F64, OP_LAND> : FpLogic<double, OP_LAND> {};
template <> struct Red<DT_F64, OP_LOR> : FpLogic<double, OP_LOR> {};
template <> struct Red<DT_BF16, OP_LAND> : Bf16Logic<OP_LAND> {};
template <> struct Red<DT_BF16, OP_LOR> : Bf16Logic<OP_LOR> {};

__device__ __forceinline__ float fused_ma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fused_ma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Compensated floating product: a pair (hi, lo) stands for hi + lo.  Each
// factor's rounding error comes back exactly from a fused multiply-add and
// gathers in lo; pairs multiply as float-float numbers.  A product that
// overflows (or is NaN) is returned as the plain product.
template <class F>
struct CompProd {
    using Acc = Pair<F>;
    static constexpr int kNA = 2;
    static __device__ __forceinline__ Acc identity() { return Acc{F(1), F(0)}; }
    static __device__ __forceinline__ void elem(Acc& a, F v) {
        const F p = a.hi * v;
        const F e = fused_ma(a.hi, v, -p);
        a.lo = fused_ma(a.lo, v, e);
        a.hi = p;
    }
    static __device__ __forceinline__ Acc combine(Acc a, Acc b) {
        const F p = a.hi * b.hi;
        if (!__builtin_isfinite(p)) return Acc{p, F(0)};
        F e = fused_ma(a.hi, b.hi, -p);
        e = fused_ma(a.hi, b.lo, e);
        e = fused_ma(a.lo, b.hi, e);
        return fast_two_sum(p, e);
    }
    static __device__ __forceinline__ F value(Acc a, F x) {
        const Acc r = combine(Acc{x, F(0)}, a);
        return __builtin_isfinite(r.hi) ? r.hi + r.lo : r.hi;
    }
};
template <> struct Red<DT_F32, OP_PROD> : CompProd<float> {
    using Out = float;
    static __device__ __forceinline__ Out finish(Acc a, Out x) { return value(a, x); }
};
template <> struct Red<DT_F64, OP_PROD> : CompProd<double> {
    using Out = double;
    static __device__ __forceinline__ Out finish(Acc a, Out x) { return value(a, x); }
};
template <> struct Red<DT_BF16, OP_PROD> : CompProd<float> {
    using Out = float;   // like bf16 sums: the fp32 accumulator
    static __device__ __forceinline__ Out finish(Acc a, Out x) { return value(a, x); }
};

}  // namespace omprt
