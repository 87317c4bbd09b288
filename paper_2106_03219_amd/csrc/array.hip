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

#include "array_kernel.h"
#include "runtime.h"

namespace omprt {

static ArrayLauncher array_launcher(int dtype, int op, bool vec, int u) {
    switch (dtype) {
        case DT_I32: return array_launcher_i32(op, vec, u);
        case DT_I64: return array_launcher_i64(op, vec, u);
        case DT_F32: return array_launcher_f32(op, vec, u);
        case DT_F64: return array_launcher_f64(op, vec, u);
        case DT_BF16: return array_launcher_bf16(op, vec, u);
    }
    return nullptr;
}

// Bytes of one private copy (the accumulator) per (dtype, op).
static int acc_bytes(int dtype, int op) {
    if (op == OP_LAND || op == OP_LOR) return 4;   // a 0/1 flag
    const bool pair = op == OP_SUM || op == OP_PROD;   // compensated (hi, lo)
    switch (dtype) {
        case DT_I32: return 4;
        case DT_I64: return 8;
        case DT_F32: return pair ? 8 : 4;
        case DT_F64: return pair ? 16 : 8;
        case DT_BF16: return pair ? 8 : 4;
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
        retire_device_memory(dev, ws.base);   // a captured graph may still name it
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
    if (!op_defined(dtype, op)) return fail(OMPRT_ERR_UNSUPPORTED, "op %d on dtype %d", op, dtype);
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
    if (!op_defined(dtype, op)) return fail(OMPRT_ERR_UNSUPPORTED, "op %d on dtype %d", op, dtype);
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
