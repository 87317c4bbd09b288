// lines.h -- per-lane runs moved through LDS one 128-byte line at a time.
//
// Under an exact static schedule a thread's iterations form one contiguous
// run per chunk, and the runs of neighbouring threads lie side by side, m/P
// (or c) elements apart.  Loading its own run, each lane of a wave touches a
// different line with every load instruction: 64 lines, 16 bytes of each,
// per instruction, and eight instructions later the same 64 lines again.
// Here a wave instead moves one line of every lane's run per pass: load
// instruction k carries lines 8k .. 8k+7 (eight lanes a line, 16 bytes
// each), so it touches eight whole lines, into a per-wave LDS buffer; then
// every lane reads its own line back and executes its iterations on it, in
// order (the lines themselves in a wave-dependent rotation, line_rot).  The
// lane that owns an iteration still executes it; the other lanes only copy
// bytes between memory and LDS.
//
// LDS layout of one buffer (64 lines, 512 16-byte slots): block b of line p
// sits in slot 8p + (b ^ line_swz(p)).  The loaders' writes are contiguous
// (instruction k, lane i -> slot 64k + i), and the owners' reads of one
// block b by 16 consecutive lanes fall on distinct banks whether LDS serves
// 16 lanes of 16 bytes (64 banks) or 8 (32 banks) per cycle.
#pragma once
#include "device.h"
#include "stream.h"

namespace omprt {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLineBytes = 128;
constexpr int kLineSlots = 8;                        // 16-byte blocks in a line
constexpr int kStageSlots = kWave * kLineSlots;      // 16-byte slots per buffer

__device__ __forceinline__ int line_swz(int p) { return (p & 7) ^ ((p >> 3) & 1); }

// Orders LDS accesses of different lanes of one wave: the LDS executes a
// wave's instructions in issue order, so only the compiler has to be kept
// from moving accesses across this point.
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Minimum over the 64 lanes of the wave (all lanes active).
__device__ __forceinline__ int64_t wave_min_i64(int64_t v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        const int64_t o = __shfl_xor(v, m, kWave);
        v = o < v ? o : v;
    }
    return v;
}

// Element offset of the 16-byte block this lane moves for line 8k + lane/8
// when lane p's line starts at element `mine` (S-byte elements).
template <int S>
__device__ __forceinline__ void line_sources(int64_t mine, int64_t (&src)[8]) {
    constexpr int PER = 16 / S;
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int p = 8 * k + (lane >> 3);
        src[k] = __shfl(mine, p, kWave) + (int64_t)PER * ((lane & 7) ^ line_swz(p));
    }
}

// Lines in a wave-dependent order.  Lane runs a multiple of 4 KiB apart
// (power-of-two chunks and team blocks) have every wave of the grid move
// lines at the same offsets at the same time, and such launches stream at
// 3.4-4.2 TB/s on gfx950 where runs at scattered offsets reach 4.7-5.0.  So
// wave g of the grid takes its lines from line (11 g) mod np on and wraps
// round: each lane still moves, and each owner still executes, the same
// lines, in rotated order.  Runs of fewer than kRotMinLines lines (strides
// under 2 KiB of fp32, where rotating measured slower) and callers that
// use the plain order keep it.
constexpr int64_t kRotMinLines = 16;

__device__ __forceinline__ int64_t line_rot(int64_t np) {
    if (np < kRotMinLines) return 0;
    const uint32_t g = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    return np <= 0x7fffffff ? (int64_t)((g * 11u) % (uint32_t)np) : (int64_t)(g * 11u);
}

// Line that pass q moves (0 <= q, rot < np); q itself in the plain order.
template <bool ROT>
__device__ __forceinline__ int64_t rot_line(int64_t q, int64_t rot, int64_t np) {
    if (!ROT) return q;
    const int64_t l = q + rot;
    return l >= np ? l - np : l;
}

// The passes q = 0 .. np-1 of a line loop whose loads run two passes ahead
// in two register sets: F provides load<S>(q) (issue the loads of pass q
// into set S) and pass<S>(q, np) (stage set S, issue pass q + 2 into it if
// q + 2 < np, then the LDS work and the stores of pass q).
template <class F>
__device__ __forceinline__ void line_passes(F& f, int64_t np) {
    if (np <= 0) return;
    f.template load<0>(0);
    if (np > 1) f.template load<1>(1);
    for (int64_t q = 0;; q += 2) {
        f.template pass<0>(q, np);
        if (q + 1 >= np) break;
        f.template pass<1>(q + 1, np);
        if (q + 2 >= np) break;
    }
}

// A wave-collective fold of np lines of the calling lane's run from element
// `mine` on (in + mine on a 128-byte boundary; np the same on every lane)
// into acc (R::kNA accumulators), through a per-wave buffer of kStageSlots
// 16-byte slots: each pass loads one line of every lane's run, eight lanes
// a line, and the owner folds its line from LDS in increasing order; the
// lines come in line_rot's order (ROT) or in increasing order; loads run
// two passes ahead (line_passes).
template <class R, int DT, bool ROT>
struct LineFold {
    using L = VecLoad<DT, 16>;
    using Vec = typename L::T;
    using S = typename DType<DT>::S;
    static_assert(sizeof(Vec) == 16, "16-byte blocks");
    static constexpr int64_t kLine = kLineBytes / (int)sizeof(S);
    const S* __restrict__ in;
    u32x4* __restrict__ buf;
    typename R::Acc* acc;
    int64_t src[8];
    int64_t np, rot;
    Vec v[2][8];

    template <int SET>
    __device__ __forceinline__ void load(int64_t q) {
        const int64_t e = rot_line<ROT>(q, rot, np) * kLine;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            v[SET][k] = L::load(reinterpret_cast<const Vec*>(in + src[k] + e));
    }
    template <int SET>
    __device__ __forceinline__ void pass(int64_t q, int64_t np) {
        const int lane = threadIdx.x & (kWave - 1);
        const int sw = line_swz(lane);
#pragma unroll
        for (int k = 0; k < 8; ++k) __builtin_memcpy(&buf[kWave * k + lane], &v[SET][k], 16);
        if (q + 2 < np) load<SET>(q + 2);
        wave_lds_order();
#pragma unroll
        for (int b = 0; b < kLineSlots; ++b) {
            const u32x4 w = buf[kLineSlots * lane + (b ^ sw)];
            Vec e;
            __builtin_memcpy(&e, &w, 16);
#pragma unroll
            for (int u = 0; u < L::PER; ++u) R::elem(acc[u % R::kNA], L::get(e, u));
        }
        wave_lds_order();
    }
};

template <class R, int DT, bool ROT = true>
__device__ __forceinline__ void line_fold(const typename DType<DT>::S* __restrict__ in,
                                          int64_t mine, int64_t np, u32x4* __restrict__ buf,
                                          typename R::Acc* acc) {
    LineFold<R, DT, ROT> f;
    f.in = in;
    f.buf = buf;
    f.acc = acc;
    f.np = np;
    f.rot = ROT ? line_rot(np) : 0;
    line_sources<(int)sizeof(typename DType<DT>::S)>(mine, f.src);
    line_passes(f, np);
}

// Start of the lines of a run [lo, hi) of S-byte elements at p: the first
// element on a 128-byte boundary (hi if none), and the number of whole
// lines from there that every lane of the wave has (wave-collective).
template <int S>
__device__ __forceinline__ void run_lines(const void* p, int64_t lo, int64_t hi, int64_t& l0,
                                          int64_t& np) {
    constexpr int64_t kLine = kLineBytes / S;
    const int64_t mis =
        (int64_t)(((reinterpret_cast<uintptr_t>(p) + (uintptr_t)(lo * S)) & (kLineBytes - 1)) / S);
    l0 = lo + ((kLine - mis) & (kLine - 1));
    if (l0 > hi) l0 = hi;
    np = wave_min_i64((hi - l0) / kLine);
}

// Host side: how many waves of a team take lines for a loop of n iterations
// over `teams` teams of `threads` threads, dist_schedule chunk dc and
// schedule chunk c (0 = none).  Chunk 0: every wave, when the smallest
// distribute block gives every lane at least one line (of `elem` bytes a
// iteration); a chunk size of at least min_chunk: the waves whose every lane
// holds a chunk of the largest block.  0 when the team is not whole waves
// or larger than max_threads.
inline int lines_waves(int64_t n, int teams, int threads, int64_t dc, int64_t c, int elem,
                       int64_t min_chunk, int max_threads) {
    if (n <= 0 || teams <= 0 || threads % kWave != 0 || threads > max_threads) return 0;
    const int64_t m_lo = dc ? (dc < n ? dc : n) : n / teams;
    const int64_t m_hi = dc ? (dc < n ? dc : n) : (n + teams - 1) / teams;
    if (c == 0) return m_lo / threads >= kLineBytes / elem ? threads / kWave : 0;
    if (c < min_chunk) return 0;
    const int64_t w = ceil_div_pos(m_hi, c) / kWave;
    return (int)(w < threads / kWave ? w : threads / kWave);
}

}  // namespace omprt
