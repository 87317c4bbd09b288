// array.hip -- array-section reduction, reduction(op: x[0:m]): every list
// item x[j] is a reduction variable of its own; iteration i of the loop
// contributes in[i*m + j] to x[j].
//
// Geometry.  The row-major block is cut into column tiles of W columns
// (W = m, whole rows, when m is small) and each tile into periods of R rows,
// with R * W <= L = threads * E * U elements (E per load, U loads in flight
// per lane).  Within a period, the element at flat offset o (row o / w, column
// o % w of the tile, w its width) belongs to lane slot (u, k) with
// o = (u * P + t) * E + k, so every lane slot keeps a private copy of one list
// item for the whole launch.  Team (c, r) takes tile c and the balanced block
// of its periods; the last row team of a tile also folds the rows left over
// after the whole periods.
//
// Combination.  The private copies go to LDS as an R x w matrix whose rows
// are folded pairwise (R -> ceil(R/2) -> ... -> 1).  With one row team per
// tile the team writes x directly.  Otherwise each team publishes its w
// partials as tagged slot words; the row teams of a tile form election
// groups, sized so that the last team of a group folds the group's rows
// with at most 16 partials per thread, and the wrap-around increment elects
// that last team.  With one group it writes x; otherwise the group results
// are published and the last group of the tile folds them and writes x.
// The last tile to finish advances the launch epoch.
#include <algorithm>
#include <map>
#include <mutex>

#include "device.h"
#include "launch.h"
#include "runtime.h"
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
    switch (u) {
        case 1: return vec ? launch_array_one<DT, OP, true, 1> : launch_array_one<DT, OP, false, 1>;
        case 2: return vec ? launch_array_one<DT, OP, true, 2> : launch_array_one<DT, OP, false, 2>;
        case 4: return vec ? launch_array_one<DT, OP, true, 4> : launch_array_one<DT, OP, false, 4>;
        case 8: return vec ? nullptr : launch_array_one<DT, OP, false, 8>;
    }
    return nullptr;
}
template <int DT>
static ArrayLauncher array_pick_op(int op, bool vec, int u) {
    switch (op) {
        case OP_SUM: return array_pick_v<DT, OP_SUM>(vec, u);
        case OP_MAX: return array_pick_v<DT, OP_MAX>(vec, u);
        case OP_MIN: return array_pick_v<DT, OP_MIN>(vec, u);
    }
    return nullptr;
}
static ArrayLauncher array_launcher(int dtype, int op, bool vec, int u) {
    switch (dtype) {
        case DT_I32: return array_pick_op<DT_I32>(op, vec, u);
        case DT_I64: return array_pick_op<DT_I64>(op, vec, u);
        case DT_F32: return array_pick_op<DT_F32>(op, vec, u);
        case DT_F64: return array_pick_op<DT_F64>(op, vec, u);
        case DT_BF16: return array_pick_op<DT_BF16>(op, vec, u);
    }
    return nullptr;
}

// Bytes of one private copy (the accumulator) per (dtype, op).
static int acc_bytes(int dtype, int op) {
    switch (dtype) {
        case DT_I32: return 4;
        case DT_I64: return 8;
        case DT_F32: return op == OP_SUM ? 8 : 4;
        case DT_F64: return op == OP_SUM ? 16 : 8;
        case DT_BF16: return op == OP_SUM ? 8 : 4;
    }
    return 16;
}

// ---------------------------------------------------------------- workspace

// Per (device, stream): a 256-byte header (done counter, epoch, status),
// the election counters (0 between launches) and the tagged slots; zeroed
// once at allocation, grown on demand (never while the stream is captured).
struct ArrayWs {
    void* base = nullptr;
    int64_t counters = 0;   // capacity, words
    int64_t words = 0;      // capacity, 64-bit slot words
    uint32_t* done() const { return static_cast<uint32_t*>(base); }
    uint32_t* epoch() const { return static_cast<uint32_t*>(base) + 16; }
    uint32_t* status() const { return static_cast<uint32_t*>(base) + 32; }
    uint32_t* ctrs() const { return reinterpret_cast<uint32_t*>(static_cast<char*>(base) + 256); }
    uint64_t* slots() const {
        return reinterpret_cast<uint64_t*>(static_cast<char*>(base) + 256 + ctr_bytes(counters));
    }
    static size_t ctr_bytes(int64_t n) { return ((size_t)n * 4 + 255) / 256 * 256; }
};
static std::mutex g_amu;
static std::map<std::pair<int, hipStream_t>, ArrayWs> g_aws;

static omprt_status array_ws_get(hipStream_t stream, int64_t counters, int64_t words,
                                 ArrayWs* out) {
    int dev = 0;
    OMPRT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_amu);
    ArrayWs& ws = g_aws[{dev, stream}];
    if (!ws.base || ws.counters < counters || ws.words < words) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        OMPRT_HIP(hipStreamIsCapturing(stream, &cs));
        if (cs != hipStreamCaptureStatusNone)
            return fail(OMPRT_ERR_INVALID,
                        "stream is being captured and its array-reduction workspace is too "
                        "small: make the same call once before capturing");
        const int64_t nc = std::max<int64_t>({counters, ws.counters, 1024});
        const int64_t nw = std::max<int64_t>({words, ws.words, (int64_t)1 << 16});
        const size_t bytes = 256 + ArrayWs::ctr_bytes(nc) + (size_t)nw * 8;
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess)
            return fail(OMPRT_ERR_NOMEM, "array workspace allocation of %zu bytes failed", bytes);
        if (ws.base) {
            OMPRT_HIP(hipStreamSynchronize(stream));
            OMPRT_HIP(hipFree(ws.base));
        }
        ws.base = p;
        ws.counters = nc;
        ws.words = nw;
        OMPRT_HIP(hipMemsetAsync(p, 0, bytes, stream));   // tags are odd: zero never matches
    }
    *out = ws;
    return OMPRT_OK;
}

void array_finalize() {
    std::lock_guard<std::mutex> lk(g_amu);
    for (auto& kv : g_aws) {
        if (!kv.second.base) continue;
        (void)hipSetDevice(kv.first.first);
        (void)hipFree(kv.second.base);
    }
    g_aws.clear();
}

uint32_t* array_status_word(int dev, hipStream_t stream) {
    std::lock_guard<std::mutex> lk(g_amu);
    auto it = g_aws.find({dev, stream});
    return (it == g_aws.end() || !it->second.base) ? nullptr : it->second.status();
}

omprt_status array_reset(int dev, hipStream_t stream) {
    std::lock_guard<std::mutex> lk(g_amu);
    auto it = g_aws.find({dev, stream});
    if (it == g_aws.end() || !it->second.base) return OMPRT_OK;
    const ArrayWs& ws = it->second;
    OMPRT_HIP(hipMemsetAsync(ws.done(), 0, 4, stream));
    OMPRT_HIP(hipMemsetAsync(ws.status(), 0, 4, stream));
    OMPRT_HIP(hipMemsetAsync(ws.ctrs(), 0, (size_t)ws.counters * 4, stream));
    return OMPRT_OK;
}

// ---------------------------------------------------------------- planning

constexpr int64_t kTileCols = 256;      // target tile width when rows are wider
constexpr int64_t kFoldItems = 16;     // partials one thread folds per election level
constexpr int kMaxLdsBytes = 64 * 1024 - 256;   // dynamic LDS; the rest is static

static int64_t gcd64(int64_t a, int64_t b) {
    while (b) { const int64_t t = a % b; a = b; b = t; }
    return a;
}

// Geometry for E elements per load; false if it cannot stream in vectors.
static bool array_geometry(int64_t rows, int64_t m, int E, int64_t L, ArrayGeom* g) {
    g->rows = rows;
    g->m = m;
    const int64_t wmax = std::min<int64_t>(kTileCols, L) / E * E;
    if (m <= wmax) {   // whole rows; a period's first element must stay 16-byte aligned
        const int64_t step = E / gcd64(m, E);
        g->W = m;
        g->R = (L / m) / step * step;
        g->col_tiles = 1;
        if (g->R < 1) return false;
    } else {           // balanced column tiles; every row start must be aligned
        if (m % E != 0) return false;
        const int64_t tiles = (m + wmax - 1) / wmax;
        g->W = ((m + tiles - 1) / tiles + E - 1) / E * E;
        g->R = L / g->W;
        const int64_t used = (m + g->W - 1) / g->W;
        if (used > INT32_MAX) return false;
        g->col_tiles = (int32_t)used;
    }
    g->np = rows / g->R;
    return true;
}

// LDS entries a team needs for its private copies: the span of a period,
// or one layer of P * E offsets when the kernel folds the U slots of a lane
// in registers (every slot live, whole rows per layer).  Maximum over the
// full tiles and the last one.
static int64_t lds_entries(const ArrayGeom& g, int64_t layer, int U) {
    const int64_t wl = g.m - (int64_t)(g.col_tiles - 1) * g.W;
    int64_t need = 0;
    for (int64_t wc : {std::min(g.W, g.m), wl}) {
        const int64_t span = g.R * wc;
        const bool fold = U > 1 && span == U * layer && layer % wc == 0;
        need = std::max(need, fold ? layer : span);
    }
    return need;
}

struct ArrayPlan {
    ArrayGeom g;
    bool vec;
    int threads, unroll;
    size_t lds;
};

static omprt_status plan_array(int64_t rows, int64_t m, int dtype, int op, const void* in,
                               const omprt_config* cfg, ArrayPlan* out) {
    const int esize = dtype_bytes(dtype);
    const int ab = acc_bytes(dtype, op);
    int P = 512, U = 4, want_teams = 0;
    bool allow_vec = true;
    if (cfg) {
        if (cfg->threads_per_team) {
            if (cfg->threads_per_team < 64 || cfg->threads_per_team > 512 ||
                cfg->threads_per_team % 64)
                return fail(OMPRT_ERR_INVALID, "threads_per_team %d", cfg->threads_per_team);
            P = cfg->threads_per_team;
        }
        if (cfg->unroll) {
            if (cfg->unroll != 1 && cfg->unroll != 2 && cfg->unroll != 4 && cfg->unroll != 8)
                return fail(OMPRT_ERR_INVALID, "unroll %d", cfg->unroll);
            U = cfg->unroll;
        }
        if (cfg->vec_bytes) {
            if (cfg->vec_bytes == esize) allow_vec = false;
            else if (cfg->vec_bytes != 16)
                return fail(OMPRT_ERR_INVALID, "vec_bytes %d (0, 16 or the element size)",
                            cfg->vec_bytes);
        }
        if (cfg->num_teams) {
            if (cfg->num_teams < 1 || cfg->num_teams > 65535)
                return fail(OMPRT_ERR_INVALID, "num_teams %d", cfg->num_teams);
            want_teams = cfg->num_teams;
        }
    }
    const bool explicit_u = cfg && cfg->unroll;
    ArrayPlan pl{};
    pl.threads = P;
    bool found = false;
    // 16-byte loads first, then element loads; the default unroll is lowered
    // until the private copies fit LDS, an explicit one is kept or dropped.
    for (int pass = allow_vec ? 0 : 1; pass < 2 && !found; ++pass) {
        const bool vec = pass == 0;
        if (vec && (reinterpret_cast<uintptr_t>(in) & 15)) continue;
        const int E = vec ? 16 / esize : 1;
        const int u0 = vec ? std::min(U, 4) : (explicit_u ? U : 8);   // element loads: 8 in flight
        for (int u = u0; u >= 1 && !found; u /= 2) {
            ArrayGeom g{};
            if (array_geometry(rows, m, E, (int64_t)P * E * u, &g)) {
                // the group fold also needs one entry per thread
                const size_t bytes =
                    (size_t)std::max<int64_t>(lds_entries(g, (int64_t)P * E, u), P) * ab;
                if (bytes <= (size_t)kMaxLdsBytes) {
                    pl.g = g;
                    pl.vec = vec;
                    pl.unroll = u;
                    pl.lds = bytes;
                    found = true;
                }
            }
            if (explicit_u) break;
        }
    }
    if (!found)
        return fail(OMPRT_ERR_INVALID,
                    "no launch geometry: the private copies of threads %d x unroll %d do not "
                    "fit %d bytes of LDS", P, U, kMaxLdsBytes);
    ArrayGeom& g = pl.g;
    // default: one team per compute unit with 16-byte loads, two with element
    // loads (which keep a quarter of the bytes in flight per lane or less)
    if (!want_teams) want_teams = device_cus() * (pl.vec ? 1 : 2);
    int64_t rt = std::max<int64_t>(1, want_teams / g.col_tiles);
    rt = std::min<int64_t>(rt, std::max<int64_t>(1, g.np));
    g.rt = (int32_t)rt;
    // Election groups: as many teams as the last one can fold with at most
    // kFoldItems partials per thread (fold_group); one group when all fit.
    const int64_t wc_max = std::min(g.W, m);
    const int64_t per_col = wc_max * 2 > P ? 1 : P / wc_max;   // threads per column
    const int64_t rounds = (wc_max + P - 1) / P;               // columns per thread
    const int64_t gs_max = std::max<int64_t>(2, kFoldItems * per_col / rounds);
    g.gs = (int32_t)std::min(rt, gs_max);
    g.ng = (int32_t)((rt + g.gs - 1) / g.gs);
    *out = pl;
    return OMPRT_OK;
}

}  // namespace omprt

using namespace omprt;

extern "C" omprt_status omprt_reduce_array(const void* d_in, int64_t rows, int64_t m,
                                           int32_t dtype, int32_t op, void* d_x,
                                           const omprt_config* cfg, void* hip_stream) {
    if (dtype < 0 || dtype >= DT_COUNT_ABI) return fail(OMPRT_ERR_UNSUPPORTED, "dtype %d", dtype);
    if (op < 0 || op >= OP_COUNT) return fail(OMPRT_ERR_UNSUPPORTED, "op %d", op);
    if (rows < 0 || m < 0) return fail(OMPRT_ERR_INVALID, "rows/m negative");
    if (m > 0 && rows > ((int64_t)1 << 50) / m)
        return fail(OMPRT_ERR_INVALID, "rows * m above 2^50");
    if (m > ((int64_t)1 << 40)) return fail(OMPRT_ERR_INVALID, "m above 2^40");
    if (rows == 0 || m == 0) return OMPRT_OK;
    if (!d_in || !d_x) return fail(OMPRT_ERR_INVALID, "in/x is NULL");
    const int esize = dtype_bytes(dtype), xsize = out_bytes(dtype, op);
    if (reinterpret_cast<uintptr_t>(d_in) % esize)
        return fail(OMPRT_ERR_INVALID, "in is not aligned to its element size");
    if (reinterpret_cast<uintptr_t>(d_x) % xsize)
        return fail(OMPRT_ERR_INVALID, "x is not aligned to its element size");
    {
        const char* ib = static_cast<const char*>(d_in);
        const char* xb = static_cast<const char*>(d_x);
        if (xb < ib + rows * m * esize && ib < xb + m * xsize)
            return fail(OMPRT_ERR_INVALID, "x overlaps in");
    }
    ArrayPlan pl;
    if (omprt_status st = plan_array(rows, m, dtype, op, d_in, cfg, &pl)) return st;
    const ArrayGeom& g = pl.g;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    ArrayCross ct{};
    if (g.rt > 1) {
        const int nw = acc_bytes(dtype, op) / 4;
        const int64_t counters = (int64_t)g.col_tiles * g.ng + (g.ng > 1 ? g.col_tiles : 0);
        const int64_t words = ((int64_t)g.rt + (g.ng > 1 ? g.ng : 0)) * m * nw;
        ArrayWs ws;
        if (omprt_status st = array_ws_get(stream, counters, words, &ws)) return st;
        ct = ArrayCross{ws.slots(), ws.slots() + (int64_t)g.rt * m * nw, ws.ctrs(), ws.done(),
                        ws.epoch(), ws.status()};
    }
    const ArrayLauncher f = array_launcher(dtype, op, pl.vec, pl.unroll);
    if (!f) return fail(OMPRT_ERR_UNSUPPORTED, "no array kernel for this combination");
    if ((int64_t)g.col_tiles * g.rt > INT32_MAX) return fail(OMPRT_ERR_INVALID, "grid too large");
    f(d_in, d_x, g, ct, pl.threads, pl.lds, stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "array launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}

extern "C" omprt_status omprt_reduce_array_plan(int64_t rows, int64_t m, int32_t dtype, int32_t op,
                                         int32_t aligned16, const omprt_config* cfg,
                                         int64_t* h_out8) {
    if (dtype < 0 || dtype >= DT_COUNT_ABI) return fail(OMPRT_ERR_UNSUPPORTED, "dtype %d", dtype);
    if (op < 0 || op >= OP_COUNT) return fail(OMPRT_ERR_UNSUPPORTED, "op %d", op);
    if (rows < 1 || m < 1) return fail(OMPRT_ERR_INVALID, "rows/m must be >= 1");
    if (!h_out8) return fail(OMPRT_ERR_INVALID, "out is NULL");
    ArrayPlan pl;
    const void* fake = reinterpret_cast<const void*>(aligned16 ? (uintptr_t)256 : (uintptr_t)260);
    if (omprt_status st = plan_array(rows, m, dtype, op, fake, cfg, &pl)) return st;
    const int64_t v[8] = {pl.g.W, pl.g.R, pl.g.col_tiles, pl.g.rt, pl.g.ng,
                          pl.vec ? 16 : dtype_bytes(dtype), pl.threads, pl.unroll};
    for (int i = 0; i < 8; ++i) h_out8[i] = v[i];
    return OMPRT_OK;
}
