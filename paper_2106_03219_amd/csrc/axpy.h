// axpy.h -- the AXPY worksharing body y[i] <- fmaf(a, x[i], y[i]) with a
// compensated sum of the updated y, as executed by one thread over the
// chunks the schedule gives it.  Shared by the static and the queue-based
// (dynamic / guided) kernels.
#pragma once
#include "device.h"
#include "lines.h"

namespace omprt {

__device__ __forceinline__ void axpy_elem(float a, const float* __restrict__ x,
                                          float* __restrict__ y, int64_t i, ff_t& acc) {
    const float r = __builtin_fmaf(a, x[i], y[i]);
    y[i] = r;
    comp_add(acc, r);
}

// Elements [lo, lo + cnt), 1 <= cnt <= B, as one batch whose loads issue
// together (one element at a time, each would wait out a memory latency):
// the missing ones load element lo + cnt - 1 again and add zero; only the
// real ones are stored.
template <int B>
__device__ __forceinline__ void axpy_batch(float a, const float* __restrict__ x,
                                           float* __restrict__ y, int64_t lo, int64_t cnt,
                                           ff_t& acc) {
    float xx[B], yy[B];
    int64_t ii[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
        ii[u] = lo + (u < cnt ? u : cnt - 1);
        xx[u] = x[ii[u]];
        yy[u] = y[ii[u]];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) yy[u] = __builtin_fmaf(a, xx[u], yy[u]);
    if (cnt == B) {   // a full batch stores unpredicated (measured faster for chunks of 4)
#pragma unroll
        for (int u = 0; u < B; ++u) y[ii[u]] = yy[u];
    } else {          // the repeats would store the same value again
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (u < cnt) y[ii[u]] = yy[u];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) comp_add(acc, u < cnt ? yy[u] : 0.0f);
}

// Elements [lo, hi) in batches of four.
__device__ __forceinline__ void axpy_elems(float a, const float* __restrict__ x,
                                           float* __restrict__ y, int64_t lo, int64_t hi,
                                           ff_t& acc) {
    for (int64_t i = lo; i < hi; i += 4) axpy_batch<4>(a, x, y, i, hi - i < 4 ? hi - i : 4, acc);
}

// Vectors [j, j + cnt), 1 <= cnt <= 8, of 16-byte aligned x and y, as one
// batch (missing vectors load the last one again, as in axpy_batch).
__device__ __forceinline__ void axpy_vbatch(float a, const float4* __restrict__ xv,
                                            float4* __restrict__ yv, int64_t j, int64_t cnt,
                                            ff_t& acc) {
    constexpr int U = 8;
    float4 xx[U], yy[U];
    int64_t jj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        jj[u] = j + (u < cnt ? u : cnt - 1);
        xx[u] = xv[jj[u]];
        yy[u] = yv[jj[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        yy[u].x = __builtin_fmaf(a, xx[u].x, yy[u].x);
        yy[u].y = __builtin_fmaf(a, xx[u].y, yy[u].y);
        yy[u].z = __builtin_fmaf(a, xx[u].z, yy[u].z);
        yy[u].w = __builtin_fmaf(a, xx[u].w, yy[u].w);
        if (u < cnt) yv[jj[u]] = yy[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool real = u < cnt;
        comp_add(acc, real ? yy[u].x : 0.0f);
        comp_add(acc, real ? yy[u].y : 0.0f);
        comp_add(acc, real ? yy[u].z : 0.0f);
        comp_add(acc, real ? yy[u].w : 0.0f);
    }
}

// A chunk [lo, hi) of at most 16 iterations that is whole 16-byte vectors of
// co-aligned x and y (chunks of 4 to 16 on an aligned block): one vector, or
// one batch of up to four, without the edge handling of longer runs --
// neighbouring lanes' chunks are adjacent, so a wave's loads cover whole
// lines.  Returns false (nothing done) for any other chunk.
__device__ __forceinline__ bool axpy_short_run(float a, const float* __restrict__ x,
                                               float* __restrict__ y, int64_t lo, int64_t hi,
                                               ff_t& acc) {
    const int64_t len = hi - lo;
    if (len < 4 || len > 16 || (len & 3) ||
        ((reinterpret_cast<uintptr_t>(x + lo) | reinterpret_cast<uintptr_t>(y + lo)) & 15))
        return false;
    if (len == 4) {
        const float4 xx = *reinterpret_cast<const float4*>(x + lo);
        float4 yy = *reinterpret_cast<const float4*>(y + lo);
        yy.x = __builtin_fmaf(a, xx.x, yy.x);
        yy.y = __builtin_fmaf(a, xx.y, yy.y);
        yy.z = __builtin_fmaf(a, xx.z, yy.z);
        yy.w = __builtin_fmaf(a, xx.w, yy.w);
        *reinterpret_cast<float4*>(y + lo) = yy;
        comp_add(acc, yy.x);
        comp_add(acc, yy.y);
        comp_add(acc, yy.z);
        comp_add(acc, yy.w);
    } else {
        axpy_vbatch(a, reinterpret_cast<const float4*>(x + lo), reinterpret_cast<float4*>(y + lo), 0,
                    len / 4, acc);
    }
    return true;
}

// One chunk [lo, hi) of the calling thread.  Where x and y are co-aligned:
// up to three elements to 16-byte alignment, vectors up to a 128-byte line
// boundary and the last up to three elements go first, as one batch; then
// whole lines -- eight 16-byte vectors of x and of y in flight per lane, so a
// lane's loads to one line issue together and the line is fetched once
// (measured at 2^26, chunk 0: 4.26 TB/s with eight, 3.65 with four, 2.91
// with sixteen); then the last vectors as one batch.  A run's edges thus cost
// two memory latencies, not four.
__device__ __forceinline__ void axpy_range(float a, const float* __restrict__ x,
                                           float* __restrict__ y, int64_t lo, int64_t hi,
                                           ff_t& acc) {
    const bool co_aligned =
        ((reinterpret_cast<uintptr_t>(x) ^ reinterpret_cast<uintptr_t>(y)) & 15) == 0;
    if (!co_aligned || hi - lo < 8) {
        axpy_elems(a, x, y, lo, hi, acc);
        return;
    }
    const uintptr_t mis = reinterpret_cast<uintptr_t>(y + lo) & 15;
    const int64_t head = (int64_t)(((16 - mis) & 15) / 4);   // 0..3 elements
    const int64_t p = lo + head;
    const int64_t nv = (hi - p) / 4;                          // >= 1 (hi - lo >= 8)
    const int64_t t0 = p + nv * 4;
    const int64_t tail = hi - t0;                             // 0..3 elements
    const float4* __restrict__ xv = reinterpret_cast<const float4*>(x + p);
    float4* __restrict__ yv = reinterpret_cast<float4*>(y + p);
    constexpr int U = 8;
    int64_t jh = (int64_t)(((128 - (reinterpret_cast<uintptr_t>(yv) & 127)) & 127) / 16);
    if (jh > nv) jh = nv;                                     // 0..7 head vectors

    if (head | jh | tail) {   // the edges, one batch; an empty group reads
                              // element lo / vector 0 (inside the run) and
                              // stores nothing
        float ex[8], ey[8];
        int64_t ei[8];
        float4 vx[U], vy[U];
        int64_t vj[U];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ei[u] = head ? lo + (u < head ? u : head - 1) : lo;
            ei[4 + u] = tail ? t0 + (u < tail ? u : tail - 1) : lo;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) vj[u] = jh ? (u < jh ? u : jh - 1) : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            ex[u] = x[ei[u]];
            ey[u] = y[ei[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            vx[u] = xv[vj[u]];
            vy[u] = yv[vj[u]];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) ey[u] = __builtin_fmaf(a, ex[u], ey[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            vy[u].x = __builtin_fmaf(a, vx[u].x, vy[u].x);
            vy[u].y = __builtin_fmaf(a, vx[u].y, vy[u].y);
            vy[u].z = __builtin_fmaf(a, vx[u].z, vy[u].z);
            vy[u].w = __builtin_fmaf(a, vx[u].w, vy[u].w);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (u < head) y[ei[u]] = ey[u];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (u < tail) y[ei[4 + u]] = ey[4 + u];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (u < jh) yv[vj[u]] = vy[u];
#pragma unroll
        for (int u = 0; u < 4; ++u) comp_add(acc, u < head ? ey[u] : 0.0f);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool real = u < jh;
            comp_add(acc, real ? vy[u].x : 0.0f);
            comp_add(acc, real ? vy[u].y : 0.0f);
            comp_add(acc, real ? vy[u].z : 0.0f);
            comp_add(acc, real ? vy[u].w : 0.0f);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) comp_add(acc, u < tail ? ey[4 + u] : 0.0f);
    }
    int64_t j = jh;
    for (; j + U <= nv; j += U) {
        float4 xx[U], yy[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xx[u] = xv[j + u];
            yy[u] = yv[j + u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            yy[u].x = __builtin_fmaf(a, xx[u].x, yy[u].x);
            yy[u].y = __builtin_fmaf(a, xx[u].y, yy[u].y);
            yy[u].z = __builtin_fmaf(a, xx[u].z, yy[u].z);
            yy[u].w = __builtin_fmaf(a, xx[u].w, yy[u].w);
            yv[j + u] = yy[u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            comp_add(acc, yy[u].x);
            comp_add(acc, yy[u].y);
            comp_add(acc, yy[u].z);
            comp_add(acc, yy[u].w);
        }
    }
    if (j < nv) axpy_vbatch(a, xv, yv, j, nv - j, acc);
}

// Chunk size 1: thread t of the block [lo, hi) executes lo + t, lo + t + P,
// ... (one-iteration chunks dealt round-robin).  A wave's lanes touch 64
// consecutive elements, so every access is coalesced and covers whole cache
// lines: the streams bypass cache residency (nontemporal), four rows in
// flight.  (Nontemporal access is a loss for the per-lane runs of larger
// chunks, whose lines are consumed by several successive loads.)
__device__ __forceinline__ void axpy_stride(float a, const float* __restrict__ x,
                                            float* __restrict__ y, int64_t lo, int64_t hi,
                                            int t, int P, ff_t& acc) {
    constexpr int U = 4;
    int64_t i = lo + t;
    for (; i + (int64_t)(U - 1) * P < hi; i += (int64_t)U * P) {
        float xx[U], yy[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xx[u] = __builtin_nontemporal_load(x + i + (int64_t)u * P);
            yy[u] = __builtin_nontemporal_load(y + i + (int64_t)u * P);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            yy[u] = __builtin_fmaf(a, xx[u], yy[u]);
            __builtin_nontemporal_store(yy[u], y + i + (int64_t)u * P);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) comp_add(acc, yy[u]);
    }
    for (; i < hi; i += P) axpy_elem(a, x, y, i, acc);
}

// Lane runs through LDS (lines.h), wave-collective: lane p owns np lines
// of 32 elements starting at element `mine` of its run (y + mine on a
// 128-byte boundary, x co-aligned with y to 16 bytes); np is the same on
// every lane.  Each pass loads one line of x and of y per lane, eight lanes
// a line, into LDS; the owner runs y[i] <- fmaf(a, x[i], y[i]) and its sum
// over its line from LDS in increasing i, and the wave stores the updated
// lines back eight lanes a line.  The lines come in line_rot's order (ROT)
// or in increasing order; loads run two passes ahead (line_passes), so a
// wave keeps 32 KiB in flight through the LDS work of a pass.
template <bool ROT>
struct AxpyLines {
    static constexpr int64_t kLine = kLineBytes / 4;
    float a;
    const float* __restrict__ x;
    float* __restrict__ y;
    f32x4* __restrict__ xs;
    f32x4* __restrict__ ys;
    ff_t* acc;
    int64_t src[8];
    int64_t np, rot;
    f32x4 vx[2][8], vy[2][8];

    template <int SET>
    __device__ __forceinline__ void load(int64_t q) {
        const int64_t l = rot_line<ROT>(q, rot, np) * kLine;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            vx[SET][k] = __builtin_nontemporal_load(
                reinterpret_cast<const f32x4*>(x + src[k] + l));
            vy[SET][k] = __builtin_nontemporal_load(
                reinterpret_cast<const f32x4*>(y + src[k] + l));
        }
    }
    template <int SET>
    __device__ __forceinline__ void pass(int64_t q, int64_t np) {
        const int lane = threadIdx.x & (kWave - 1);
        const int sw = line_swz(lane);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            xs[kWave * k + lane] = vx[SET][k];
            ys[kWave * k + lane] = vy[SET][k];
        }
        if (q + 2 < np) load<SET>(q + 2);
        wave_lds_order();
#pragma unroll
        for (int b = 0; b < kLineSlots; ++b) {
            const int slot = kLineSlots * lane + (b ^ sw);
            const f32x4 xx = xs[slot];
            f32x4 yy = ys[slot];
            yy.x = __builtin_fmaf(a, xx.x, yy.x);
            yy.y = __builtin_fmaf(a, xx.y, yy.y);
            yy.z = __builtin_fmaf(a, xx.z, yy.z);
            yy.w = __builtin_fmaf(a, xx.w, yy.w);
            ys[slot] = yy;
            comp_add(*acc, yy.x);
            comp_add(*acc, yy.y);
            comp_add(*acc, yy.z);
            comp_add(*acc, yy.w);
        }
        wave_lds_order();
        const int64_t l = rot_line<ROT>(q, rot, np) * kLine;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            __builtin_nontemporal_store(ys[kWave * k + lane],
                                        reinterpret_cast<f32x4*>(y + src[k] + l));
        wave_lds_order();
    }
};

template <bool ROT>
__device__ __forceinline__ void axpy_lines(float a, const float* __restrict__ x,
                                           float* __restrict__ y, int64_t mine, int64_t np,
                                           f32x4* __restrict__ xs, f32x4* __restrict__ ys,
                                           ff_t& acc) {
    AxpyLines<ROT> f;
    f.a = a;
    f.x = x;
    f.y = y;
    f.xs = xs;
    f.ys = ys;
    f.acc = &acc;
    f.np = np;
    f.rot = ROT ? line_rot(np) : 0;
    line_sources<4>(mine, f.src);
    line_passes(f, np);
}

// One run [lo, hi) of the calling lane, wave-collective (every lane of the
// wave calls it, with its own run): the part before y's next line boundary
// and the part after as many whole lines as every lane of the wave has, by
// the lane alone, then those whole lines through axpy_lines.  Both edges go
// first: a run's last partial line is the next lane's first, and taken at
// the same time the two halves share one fetch of the line (with the tail
// after the lines, guided rounds ran 1-5 % slower).  A lane's iterations
// stay in increasing order within each edge and line; the lines come in
// line_rot's order (ROT) or in increasing order.
template <bool ROT = true>
__device__ __forceinline__ void axpy_run_lines(float a, const float* __restrict__ x,
                                               float* __restrict__ y, int64_t lo, int64_t hi,
                                               f32x4* __restrict__ xs, f32x4* __restrict__ ys,
                                               ff_t& acc) {
    int64_t l0, np;
    run_lines<4>(y, lo, hi, l0, np);
    const int64_t r = l0 + np * (kLineBytes / 4);
    if (l0 > lo) axpy_range(a, x, y, lo, l0, acc);
    if (r < hi) axpy_range(a, x, y, r, hi, acc);
    axpy_lines<ROT>(a, x, y, l0, np, xs, ys, acc);
}

// Runs of the 64 lanes of a wave that lie side by side in lane order (lane
// l's run ends where lane l + 1's starts), moved as one union [ulo, uhi):
// pass q holds 64 consecutive 128-byte lines of the union (instruction k,
// lane i moves block (i & 7) ^ line_swz(p) of line p = 8k + i/8, the LDS
// layout of AxpyLines), and every lane executes the elements of its own run
// that the pass holds, from LDS, in increasing order.  Blocks wholly inside
// the union move as 16-byte vectors, the union's first and last blocks
// element by element; nothing outside it is read or written.  For short
// runs (a pass holds 2048 elements: with runs of r elements about 2048 / r
// lanes compute in it), whatever their alignment: no lane has edges of its
// own.  Loads run two passes ahead (line_passes).  AXPY false: the fold of
// the sum alone (y read, the owner adding its elements; nothing stored).
template <bool AXPY>
struct AxpyUnionT {
    static constexpr int64_t kLine = kLineBytes / 4;
    static constexpr int64_t kPass = kLine * kWave;   // elements a pass holds
    float a;
    const float* __restrict__ x;
    float* __restrict__ y;
    f32x4* __restrict__ xs;
    f32x4* __restrict__ ys;
    ff_t* acc;
    // offsets in elements from x + u0 / y + u0, the first element of the
    // union's first line (the union of short runs spans under 2^31)
    int32_t ulo, uhi;   // the union
    int32_t lo, hi;     // this lane's run
    int32_t src[8];     // the block this lane moves in pass 0, instruction k
    f32x4 vx[2][8], vy[2][8];

    template <int SET>
    __device__ __forceinline__ void load(int64_t q) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int32_t e = (int32_t)q * (int32_t)kPass + src[k];
            if (e >= ulo && e + 4 <= uhi) {
                if (AXPY)
                    vx[SET][k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(x + e));
                vy[SET][k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(y + e));
            } else if (e + 4 > ulo && e < uhi) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (e + u >= ulo && e + u < uhi) {
                        if (AXPY) vx[SET][k][u] = x[e + u];
                        vy[SET][k][u] = y[e + u];
                    }
            }
        }
    }
    template <int SET>
    __device__ __forceinline__ void pass(int64_t q, int64_t np) {
        const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (AXPY) xs[kWave * k + lane] = vx[SET][k];
            ys[kWave * k + lane] = vy[SET][k];
        }
        if (q + 2 < np) load<SET>(q + 2);
        wave_lds_order();
        const int32_t w0 = (int32_t)q * (int32_t)kPass;
        const int r0 = (lo > w0 ? lo : w0) - w0;
        const int r1 = (hi < w0 + (int32_t)kPass ? hi : w0 + (int32_t)kPass) - w0;
        auto slot_of = [](int r) {
            const int pl = r >> 5;
            return kLineSlots * pl + (((r >> 2) & 7) ^ line_swz(pl));
        };
        auto one = [&](int r) {
            float* yf = reinterpret_cast<float*>(ys + slot_of(r));
            if (AXPY) {
                const float* xf = reinterpret_cast<const float*>(xs + slot_of(r));
                const float v = __builtin_fmaf(a, xf[r & 3], yf[r & 3]);
                yf[r & 3] = v;
                comp_add(*acc, v);
            } else {
                comp_add(*acc, yf[r & 3]);
            }
        };
        auto block = [&](f32x4& yy, const f32x4& xx) {
            if (AXPY) {
#pragma unroll
                for (int u = 0; u < 4; ++u) yy[u] = __builtin_fmaf(a, xx[u], yy[u]);
            }
        };
        // the lane's elements of the pass: up to a 16-byte block boundary one
        // by one, then whole blocks (two loaded ahead of their use), then the rest
        int r = r0;
        for (; r < r1 && (r & 3); ++r) one(r);
        for (; r + 8 <= r1; r += 8) {
            const int sa = slot_of(r), sb = slot_of(r + 4);
            f32x4 xa = {}, xb = {};
            if (AXPY) {
                xa = xs[sa];
                xb = xs[sb];
            }
            f32x4 ya = ys[sa], yb = ys[sb];
            block(ya, xa);
            block(yb, xb);
            if (AXPY) {
                ys[sa] = ya;
                ys[sb] = yb;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) comp_add(*acc, ya[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) comp_add(*acc, yb[u]);
        }
        for (; r + 4 <= r1; r += 4) {
            const int sa = slot_of(r);
            f32x4 xa = {};
            if (AXPY) xa = xs[sa];
            f32x4 ya = ys[sa];
            block(ya, xa);
            if (AXPY) ys[sa] = ya;
#pragma unroll
            for (int u = 0; u < 4; ++u) comp_add(*acc, ya[u]);
        }
        for (; r < r1; ++r) one(r);
        wave_lds_order();
        if (AXPY) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int32_t e = w0 + src[k];
                const f32x4 v = ys[kWave * k + lane];
                if (e >= ulo && e + 4 <= uhi) {
                    __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(y + e));
                } else if (e + 4 > ulo && e < uhi) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (e + u >= ulo && e + u < uhi) y[e + u] = v[u];
                }
            }
            wave_lds_order();
        }
    }
};
using AxpyUnion = AxpyUnionT<true>;

// One run [lo, hi) of the calling lane, wave-collective: through AxpyUnion
// when the wave's runs lie side by side (as the static schedules' rounds
// do), else the lane alone.
constexpr int64_t kUnionRun = 128;   // the longest runs the union path is for
template <bool AXPY = true>
__device__ __forceinline__ void axpy_union_lines(float a, const float* __restrict__ x,
                                                 float* __restrict__ y, int64_t lo, int64_t hi,
                                                 f32x4* __restrict__ xs, f32x4* __restrict__ ys,
                                                 ff_t* acc);
__device__ __forceinline__ void axpy_run_union(float a, const float* __restrict__ x,
                                               float* __restrict__ y, int64_t lo, int64_t hi,
                                               f32x4* __restrict__ xs, f32x4* __restrict__ ys,
                                               ff_t& acc) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t next_lo = __shfl_down(lo, 1, kWave);
    const bool joined = lane == kWave - 1 || hi == next_lo;
    if (__ballot(joined) != ~0ull) {
        axpy_range(a, x, y, lo, hi, acc);
        return;
    }
    axpy_union_lines(a, x, y, lo, hi, xs, ys, &acc);
}

// The union of the wave's runs through AxpyUnionT (the runs lie side by side).
template <bool AXPY>
__device__ __forceinline__ void axpy_union_lines(float a, const float* __restrict__ x,
                                                 float* __restrict__ y, int64_t lo, int64_t hi,
                                                 f32x4* __restrict__ xs, f32x4* __restrict__ ys,
                                                 ff_t* acc) {
    const int lane = threadIdx.x & (kWave - 1);
    AxpyUnionT<AXPY> f;
    f.a = a;
    f.xs = xs;
    f.ys = ys;
    f.acc = acc;
    const int64_t ulo = __shfl(lo, 0, kWave), uhi = __shfl(hi, kWave - 1, kWave);
    const int64_t u0 = ulo - (int64_t)((reinterpret_cast<uintptr_t>(y + ulo) & (kLineBytes - 1)) / 4);
    f.x = AXPY ? x + u0 : x;
    f.y = y + u0;
    f.lo = (int32_t)(lo - u0);
    f.hi = (int32_t)(hi - u0);
    f.ulo = (int32_t)(ulo - u0);
    f.uhi = (int32_t)(uhi - u0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int pl = 8 * k + (lane >> 3);
        f.src[k] = (int32_t)(AxpyUnionT<AXPY>::kLine * pl + 4 * ((lane & 7) ^ line_swz(pl)));
    }
    const int64_t nlines = (uhi - u0 + AxpyUnionT<AXPY>::kLine - 1) / AxpyUnionT<AXPY>::kLine;
    line_passes(f, (nlines + kWave - 1) / kWave);
}

// End of the region: the team tree, the cross-team publish and last-team
// election, and sum[0] <- sum[0] + the launch's total (compensated).
// epoch was read at the start of the kernel (when gridDim.x > 1).
__device__ __forceinline__ void axpy_finish_sum(ff_t acc, float* __restrict__ sum,
                                                const CrossTeam& ct, uint32_t epoch,
                                                ff_t* lds_slots, int* s_last) {
    using R = Red<DT_F32, OP_SUM>;
    const int64_t T = gridDim.x;
    const int t = threadIdx.x;
    acc = team_reduce<R>(acc, lds_slots);
    if (T == 1) {
        if (t == 0) sum[0] = R::finish(acc, sum[0]);
        return;
    }
    const uint32_t tag = launch_tag(epoch);
    if (!publish_and_elect(acc, ct.slots + (size_t)blockIdx.x * kSlotWords, ct.counter,
                           (uint32_t)(T - 1), tag, s_last))
        return;
    const ff_t cmb = combine_slots<R>(ct.slots, T, tag, ct.status, lds_slots);
    if (t == 0) {
        sum[0] = R::finish(cmb, sum[0]);
        advance_epoch(ct.epoch, epoch);
    }
}

}  // namespace omprt
