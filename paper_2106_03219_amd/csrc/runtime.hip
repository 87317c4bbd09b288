// runtime.hip -- host runtime and C-ABI entry points for the plain paths:
// static-schedule bounds, workspaces, configuration resolution, and the
// reduce / static-map / AXPY / empty-region launches.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "launch.h"
#include "runtime.h"
#include "sched.h"

namespace omprt {

// ---------------------------------------------------------------- errors

static thread_local std::string t_err;

omprt_status fail(omprt_status st, const char* fmt, ...) {
    char buf[2048];   // room for a compiler log excerpt
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return st;
}

omprt_status ok() { return OMPRT_OK; }

int dtype_bytes(int dtype) {
    switch (dtype) {
        case OMPRT_I32: case OMPRT_F32: return 4;
        case OMPRT_I64: case OMPRT_F64: return 8;
        case OMPRT_BF16: return 2;
    }
    return 0;
}

int out_bytes(int dtype, int op) {
    if (dtype == OMPRT_BF16 && (op == OMPRT_SUM || op == OMPRT_PROD)) return 4;   // fp32 accumulator
    return dtype_bytes(dtype);
}

// ---------------------------------------------------------------- workspaces

static std::mutex g_mu;
static std::map<std::pair<int, hipStream_t>, Workspace> g_ws;   // node addresses are stable
static std::atomic<uint64_t> g_ws_generation{1};                // bumped when workspaces are freed

static std::mutex g_retire_mu;
static std::vector<std::pair<int, void*>> g_retired;

void retire_device_memory(int dev, void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_retire_mu);
    g_retired.emplace_back(dev, p);
}

static void free_retired() {
    std::lock_guard<std::mutex> lk(g_retire_mu);
    for (auto& r : g_retired) {
        (void)hipSetDevice(r.first);
        (void)hipFree(r.second);
    }
    g_retired.clear();
}

// Last workspace this host thread used: a repeat call on the same stream
// skips the lock and the map (a stream is never shared between threads).
struct WsMemo {
    int dev = -1;
    hipStream_t stream = nullptr;
    Workspace* ws = nullptr;
    uint64_t generation = 0;
};
static thread_local WsMemo t_ws;

omprt_status workspace_get(hipStream_t stream, int32_t teams, Workspace** out) {
    int dev = 0;
    OMPRT_HIP(hipGetDevice(&dev));
    if (t_ws.ws && t_ws.dev == dev && t_ws.stream == stream &&
        t_ws.generation == g_ws_generation.load(std::memory_order_acquire) &&
        t_ws.ws->capacity >= teams) {
        *out = t_ws.ws;
        return OMPRT_OK;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace& ws = g_ws[{dev, stream}];
    if (ws.capacity < teams) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        OMPRT_HIP(hipStreamIsCapturing(stream, &cs));
        if (cs != hipStreamCaptureStatusNone)
            return fail(OMPRT_ERR_INVALID,
                        "stream is being captured and its workspace holds %d team slots "
                        "(%d needed): call omprt_workspace_reserve before capturing",
                        ws.capacity, teams);
        const int32_t cap = std::max<int32_t>(teams, 4096);
        void* p = nullptr;
        if (hipMalloc(&p, 256 + (size_t)cap * kSlotBytes) != hipSuccess)
            return fail(OMPRT_ERR_NOMEM, "workspace allocation of %d slots failed", cap);
        // earlier launches, and graphs a caller captured, may still use the old one
        retire_device_memory(dev, ws.base);
        ws.base = p;
        ws.capacity = cap;
        // header and slots, once: tags are odd, so zeroed slots never match
        OMPRT_HIP(hipMemsetAsync(p, 0, 256 + (size_t)cap * kSlotBytes, stream));
    }
    t_ws = WsMemo{dev, stream, &ws, g_ws_generation.load(std::memory_order_acquire)};
    *out = &ws;
    return OMPRT_OK;
}

// ---------------------------------------------------------------- configuration

struct TuneKey {
    int dtype, op, body, log2n;
    bool operator<(const TuneKey& o) const {
        return std::tie(dtype, op, body, log2n) < std::tie(o.dtype, o.op, o.body, o.log2n);
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, LaunchCfg> g_tune;

static int floor_log2(int64_t n) {
    int l = 0;
    while (n > 1) { n >>= 1; ++l; }
    return l;
}

int device_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cached[dev] = cus;
    }
    return cached[dev];
}

// Built-in choice for reductions: 512 threads, 16-byte loads, 4 in flight
// per lane, one team per CU for large inputs (fewer, longer team blocks
// measured fastest on gfx950: 6.97 TB/s fp32, 7.11 TB/s int64 at 2^28) and
// one team per 32 KiB of input (one unrolled sweep) below that.  The AXPY
// body (body 1; body 2 is the AXPY-then-sum region) keeps 256 threads and
// up to 8 teams per CU, except for user chunks (2^26 fp32 on gfx950): the
// AXPY's chunk 1 takes one team of 512 threads per CU (5.35 TB/s against
// 4.95 with 8 teams of 256; the region's stays at 6.0 with the latter), and
// chunks of more than 512 iterations take 512 threads and about 128 chunks
// a team (chunk 1024: 5.0 against 3.1 TB/s, chunk 768 5.3 against 3.5, with
// 8 teams of 256 a CU, whose blocks of 32768 iterations hold less than a
// wave's worth of such chunks; up to 512 the two launches run alike), the
// team count rounded down to whole rounds of resident teams (one such team
// a CU: 263 teams for chunk 2000 ran a second round for 7 teams, 3.1
// against 4.8 TB/s with 256); with fewer than two waves' worth of chunks a
// CU, the waves that hold chunks spread over all CUs (chunk 4096: 256 teams
// of 64 threads, 4.3 against 3.8 TB/s with 128 teams of 512).
static LaunchCfg heuristic(int64_t n, int dtype, int body, int64_t chunk) {
    LaunchCfg c = body ? LaunchCfg{0, 256, 16, 4} : LaunchCfg{0, 512, 16, 4};
    const int64_t bytes = n * (body ? 12 : dtype_bytes(dtype));
    const int64_t per = (int64_t)c.threads * c.vec * c.unroll;
    int64_t t = (bytes + per - 1) / per;
    const int64_t cus = device_cus();
    int64_t cap = body ? 8 * cus : cus;
    if (body == 1 && chunk == 1) {
        c.threads = 512;
        cap = cus;
    } else if (body && chunk > 512) {
        constexpr int64_t kLanes = 64;                                          // a wave
        const int64_t waves = ((n + chunk - 1) / chunk + kLanes - 1) / kLanes;  // waves of chunks
        if (waves >= 2 * cus) {
            c.threads = 512;
            t = (n + 128 * chunk - 1) / (128 * chunk);
            t = t / cus * cus;
        } else {
            t = std::min(waves, cus);
            c.threads = (int)(kLanes * std::min<int64_t>((waves + t - 1) / t, 8));
        }
    }
    t = std::min<int64_t>(std::max<int64_t>(t, 1), cap);
    c.teams = (int)t;
    return c;
}

static bool valid_threads(int t) { return t >= 64 && t <= 1024 && t % 64 == 0; }

// Largest trip count accepted (keeps every byte offset far from int64 overflow).
constexpr int64_t kMaxTrip = (int64_t)1 << 50;

omprt_status resolve_config(int64_t n, int dtype, int op, int body, int64_t chunk,
                            const omprt_config* cfg, LaunchCfg* out, int* source) {
    if (cfg) {
        if (cfg->tile_kib != 0 && (cfg->tile_kib < 4 || cfg->tile_kib > 65536))
            return fail(OMPRT_ERR_INVALID, "tile_kib %d outside 4..65536", cfg->tile_kib);
        if (cfg->num_teams < 0 || cfg->num_teams > 65535)
            return fail(OMPRT_ERR_INVALID, "num_teams %d outside 0..65535", cfg->num_teams);
        if (cfg->threads_per_team != 0 && !valid_threads(cfg->threads_per_team))
            return fail(OMPRT_ERR_INVALID, "threads_per_team %d: need 64..1024 step 64",
                        cfg->threads_per_team);
        if (cfg->vec_bytes != 0 && cfg->vec_bytes != 8 && cfg->vec_bytes != 16)
            return fail(OMPRT_ERR_INVALID, "vec_bytes %d: need 0, 8 or 16", cfg->vec_bytes);
        if (cfg->unroll != 0 && cfg->unroll != 1 && cfg->unroll != 2 && cfg->unroll != 4 &&
            cfg->unroll != 8)
            return fail(OMPRT_ERR_INVALID, "unroll %d: need 0, 1, 2, 4 or 8", cfg->unroll);
    }
    const bool full = cfg && cfg->num_teams && cfg->threads_per_team && cfg->vec_bytes &&
                      cfg->unroll;
    LaunchCfg base{};
    int src = kSrcExplicit;
    if (!full) {
        bool have = false;
        // the picker and the tuned cache know the sum / max / min kernels only
        if (op <= OMPRT_MIN && !(cfg && (cfg->flags & OMPRT_CFG_NO_MODEL))) {
            have = model_pick(n, dtype, op, body ? 1 : 0, chunk, &base);
            if (have) src = kSrcModel;
        }
        if (!have && op <= OMPRT_MIN) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune.find(TuneKey{dtype, op, body ? 1 : 0, floor_log2(n)});
            if (it != g_tune.end()) {
                base = it->second;
                have = true;
                src = kSrcTuned;
            }
        }
        if (!have) {
            base = heuristic(n, dtype, body, chunk);
            src = kSrcHeuristic;
        }
    }
    if (cfg) {
        if (cfg->num_teams) base.teams = cfg->num_teams;
        if (cfg->threads_per_team) base.threads = cfg->threads_per_team;
        if (cfg->vec_bytes) base.vec = cfg->vec_bytes;
        if (cfg->unroll) base.unroll = cfg->unroll;
    }
    *out = base;
    if (source) *source = src;
    return OMPRT_OK;
}

// ---------------------------------------------------------------- schedule checks

omprt_status check_sched(const omprt_sched* s, bool allow_auto) {
    if (!s) return fail(OMPRT_ERR_INVALID, "schedule pointer is NULL");
    if (s->n < 0 || s->n > kMaxTrip)
        return fail(OMPRT_ERR_INVALID, "n = %lld outside 0..2^50", (long long)s->n);
    const int lo = allow_auto ? 0 : 1;
    if (s->num_teams < lo)
        return fail(OMPRT_ERR_INVALID, "num_teams = %d < %d", s->num_teams, lo);
    if (s->threads_per_team < lo || s->threads_per_team > 1024)
        return fail(OMPRT_ERR_INVALID, "threads_per_team = %d outside %d..1024",
                    s->threads_per_team, lo);
    if (s->dist_chunk < 0 || s->chunk < 0)
        return fail(OMPRT_ERR_INVALID, "negative chunk size");
    return OMPRT_OK;
}

static omprt_status check_member(const omprt_sched* s, int32_t team, int32_t thread) {
    if (omprt_status st = check_sched(s, false)) return st;
    if (team < 0 || team >= s->num_teams)
        return fail(OMPRT_ERR_INVALID, "team %d outside 0..%d", team, s->num_teams - 1);
    if (thread < 0 || thread >= s->threads_per_team)
        return fail(OMPRT_ERR_INVALID, "thread %d outside 0..%d", thread,
                    s->threads_per_team - 1);
    return OMPRT_OK;
}

// Per-thread chunk layout: the team's blocks are full (dist_chunk
// iterations) except possibly its last one, which can be the loop's partial
// final block; a full block gives the thread `f` chunks, the partial one `g`.
struct ThreadLayout {
    int64_t nb;        // team blocks
    int64_t f;         // chunks per full block (or in the only block if dc == 0)
    int64_t g;         // chunks in the last block when it is partial
    bool last_partial;
};

static ThreadLayout layout(const omprt_sched* s, int64_t k, int64_t t) {
    ThreadLayout L{};
    const int64_t n = s->n, T = s->num_teams, P = s->threads_per_team;
    L.nb = team_nblocks(n, T, s->dist_chunk, k);
    if (L.nb == 0) return L;
    if (s->dist_chunk == 0) {
        const Range b = team_block(n, T, 0, k, 0);
        L.f = thread_nchunks(b.hi - b.lo, P, s->chunk, t);
        return L;
    }
    const Range last = team_block(n, T, s->dist_chunk, k, L.nb - 1);
    L.f = thread_nchunks(s->dist_chunk, P, s->chunk, t);
    L.last_partial = (last.hi - last.lo) < s->dist_chunk;
    if (L.last_partial) L.g = thread_nchunks(last.hi - last.lo, P, s->chunk, t);
    return L;
}

}  // namespace omprt

using namespace omprt;

// ---------------------------------------------------------------- C ABI: bounds

extern "C" omprt_status omprt_sched_count(const omprt_sched* s, int32_t team, int32_t thread,
                                          int64_t* n_chunks, int64_t* n_iters) {
    if (omprt_status st = check_member(s, team, thread)) return st;
    if (!n_chunks || !n_iters) return fail(OMPRT_ERR_INVALID, "output pointer is NULL");
    const ThreadLayout L = layout(s, team, thread);
    const int64_t P = s->threads_per_team;
    int64_t chunks = 0, iters = 0;
    if (L.nb > 0) {
        const int64_t full_blocks = L.last_partial ? L.nb - 1 : L.nb;
        chunks = full_blocks * L.f + (L.last_partial ? L.g : 0);
        auto share = [&](int64_t m) -> int64_t { return thread_niters(m, P, s->chunk, thread); };
        if (s->dist_chunk == 0) {
            const Range b = team_block(s->n, s->num_teams, 0, team, 0);
            iters = share(b.hi - b.lo);
        } else {
            iters = full_blocks * share(s->dist_chunk);
            if (L.last_partial) {
                const Range b = team_block(s->n, s->num_teams, s->dist_chunk, team, L.nb - 1);
                iters += share(b.hi - b.lo);
            }
        }
    }
    *n_chunks = chunks;
    *n_iters = iters;
    return OMPRT_OK;
}

extern "C" omprt_status omprt_for_static_bounds(const omprt_sched* s, int32_t team,
                                                int32_t thread, int64_t j, int64_t* lb,
                                                int64_t* ub, int32_t* is_last) {
    if (omprt_status st = check_member(s, team, thread)) return st;
    if (!lb || !ub || !is_last) return fail(OMPRT_ERR_INVALID, "output pointer is NULL");
    if (j < 0) return fail(OMPRT_ERR_INVALID, "chunk index %lld < 0", (long long)j);
    const ThreadLayout L = layout(s, team, thread);
    const int64_t n = s->n, T = s->num_teams, P = s->threads_per_team;
    *lb = *ub = n;
    *is_last = 0;
    if (L.nb == 0) return OMPRT_OK;
    const int64_t full_blocks = L.last_partial ? L.nb - 1 : L.nb;
    int64_t bi, jj;
    if (L.f > 0 && j < full_blocks * L.f) {
        bi = j / L.f;
        jj = j - bi * L.f;
    } else if (L.last_partial && j - full_blocks * L.f < L.g) {
        bi = L.nb - 1;
        jj = j - full_blocks * L.f;
    } else {
        return OMPRT_OK;   // past the thread's last chunk
    }
    const Range b = team_block(n, T, s->dist_chunk, team, bi);
    const Range c = thread_chunk(b.lo, b.hi - b.lo, P, s->chunk, thread, jj);
    *lb = c.lo;
    *ub = c.hi;
    *is_last = (c.lo < c.hi && c.hi == n) ? 1 : 0;
    return OMPRT_OK;
}

// ---------------------------------------------------------------- C ABI: launches

static omprt_status check_ptr_align(const void* p, int bytes, const char* what) {
    if (reinterpret_cast<uintptr_t>(p) % (uintptr_t)bytes != 0)
        return fail(OMPRT_ERR_INVALID, "%s is not %d-byte aligned", what, bytes);
    return OMPRT_OK;
}

extern "C" omprt_status omprt_reduce(const void* d_in, int64_t n, int32_t dtype, int32_t op,
                                     void* d_x, const omprt_config* cfg, void* hip_stream) {
    if (dtype < 0 || dtype >= DT_COUNT_ABI) return fail(OMPRT_ERR_UNSUPPORTED, "dtype %d", dtype);
    if (!op_defined(dtype, op)) return fail(OMPRT_ERR_UNSUPPORTED, "op %d on dtype %d", op, dtype);
    if (n < 0 || n > kMaxTrip)
        return fail(OMPRT_ERR_INVALID, "n = %lld outside 0..2^50", (long long)n);
    if (!d_x) return fail(OMPRT_ERR_INVALID, "x is NULL");
    if (n > 0 && !d_in) return fail(OMPRT_ERR_INVALID, "input is NULL with n > 0");
    if (omprt_status st = check_ptr_align(d_in, dtype_bytes(dtype), "input")) return st;
    if (omprt_status st = check_ptr_align(d_x, out_bytes(dtype, op), "x")) return st;
    LaunchCfg lc;
    if (omprt_status st = resolve_config(n, dtype, op, 0, -1, cfg, &lc, nullptr)) return st;
    if (n == 0) return OMPRT_OK;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    Workspace* ws = nullptr;
    if (omprt_status st = workspace_get(stream, lc.teams, &ws)) return st;
    const bool exact = cfg && (cfg->flags & OMPRT_CFG_EXACT_THREAD_MAP);
    if (exact && op > OMPRT_MIN)
        return fail(OMPRT_ERR_UNSUPPORTED, "EXACT_THREAD_MAP takes sum, max and min");
    const hipError_t e =
        exact ? launch_reduce_exact(dtype, op, d_in, n, d_x, lc.teams, lc.threads, ws->cross(), stream)
              : launch_reduce(dtype, op, lc.vec, lc.unroll, d_in, n, d_x, lc.teams, lc.threads,
                              ws->cross(), stream);
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "reduce launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}

extern "C" omprt_status omprt_static_map(const omprt_sched* s, int32_t* d_owner,
                                         uint32_t* d_count, void* hip_stream) {
    if (omprt_status st = check_sched(s, false)) return st;
    if ((int64_t)s->num_teams * s->threads_per_team > INT32_MAX)
        return fail(OMPRT_ERR_INVALID, "num_teams * threads_per_team exceeds int32 owner ids");
    if (s->n == 0) return OMPRT_OK;
    if (!d_owner || !d_count) return fail(OMPRT_ERR_INVALID, "owner/count is NULL");
    const hipError_t e = launch_static_map(s->n, s->num_teams, s->threads_per_team, s->dist_chunk,
                                           s->chunk, d_owner, d_count,
                                           static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "map launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}

extern "C" omprt_status omprt_axpy_sum(float a, const float* d_x, float* d_y, float* d_sum,
                                       const omprt_sched* s, const omprt_config* cfg,
                                       void* hip_stream) {
    if (omprt_status st = check_sched(s, true)) return st;
    if (!d_sum) return fail(OMPRT_ERR_INVALID, "sum is NULL");
    if (s->n > 0 && (!d_x || !d_y)) return fail(OMPRT_ERR_INVALID, "x/y is NULL with n > 0");
    if (omprt_status st = check_ptr_align(d_x, 4, "x")) return st;
    if (omprt_status st = check_ptr_align(d_y, 4, "y")) return st;
    if (omprt_status st = check_ptr_align(d_sum, 4, "sum")) return st;
    if (s->n > 0) {
        const char* xb = reinterpret_cast<const char*>(d_x);
        const char* yb = reinterpret_cast<const char*>(d_y);
        if (xb < yb + s->n * 4 && yb < xb + s->n * 4)
            return fail(OMPRT_ERR_INVALID, "x and y overlap");
    }
    LaunchCfg lc;
    if (omprt_status st = resolve_config(s->n, OMPRT_F32, OMPRT_SUM, 1, s->chunk, cfg, &lc, nullptr))
        return st;
    const int teams = s->num_teams ? s->num_teams : lc.teams;
    if (teams > 65535)
        return fail(OMPRT_ERR_INVALID, "num_teams %d above 65535 (cross-team slot limit)", teams);
    const int threads = s->threads_per_team ? s->threads_per_team : lc.threads;
    if (s->n == 0) return OMPRT_OK;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    Workspace* ws = nullptr;
    if (omprt_status st = workspace_get(stream, teams, &ws)) return st;
    const hipError_t e = launch_axpy_sum(a, d_x, d_y, d_sum, s->n, teams, threads, s->dist_chunk,
                                         s->chunk, ws->cross(), stream);
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "axpy launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}

extern "C" omprt_status omprt_empty_region(const omprt_sched* s, int64_t* d_iters,
                                           void* hip_stream) {
    if (omprt_status st = check_sched(s, false)) return st;
    if (s->num_teams > 65535)
        return fail(OMPRT_ERR_INVALID, "num_teams %d above 65535 (cross-team slot limit)",
                    s->num_teams);
    if (omprt_status st = check_ptr_align(d_iters, 8, "iters")) return st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    Workspace* ws = nullptr;
    if (omprt_status st = workspace_get(stream, s->num_teams, &ws)) return st;
    const hipError_t e = launch_empty_region(s->n, s->num_teams, s->threads_per_team,
                                             s->dist_chunk, s->chunk, d_iters, ws->cross(), stream);
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "empty launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}

// ---------------------------------------------------------------- C ABI: configuration

extern "C" omprt_status omprt_resolve_config(int64_t n, int32_t dtype, int32_t op, int32_t body,
                                             int64_t chunk, const omprt_config* cfg,
                                             omprt_config* out, int32_t* source) {
    if (!out) return fail(OMPRT_ERR_INVALID, "out is NULL");
    if (dtype < 0 || dtype >= DT_COUNT_ABI || op < 0 || op > 2 || body < 0 || body > 1)
        return fail(OMPRT_ERR_INVALID, "bad dtype/op/body");
    LaunchCfg lc;
    int src = 0;
    if (omprt_status st = resolve_config(n, dtype, op, body, chunk, cfg, &lc, &src)) return st;
    memset(out, 0, sizeof *out);
    out->num_teams = lc.teams;
    out->threads_per_team = lc.threads;
    out->vec_bytes = lc.vec;
    out->unroll = lc.unroll;
    if (source) *source = src;
    return OMPRT_OK;
}

extern "C" omprt_status omprt_tune_set(int32_t dtype, int32_t op, int32_t body, int32_t log2n,
                                       const omprt_config* cfg) {
    if (dtype < 0 || dtype >= DT_COUNT_ABI || op < 0 || op > 2 || body < 0 || body > 1 ||
        log2n < 0 || log2n > 62)
        return fail(OMPRT_ERR_INVALID, "bad tune key");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!cfg) {
        g_tune.erase(TuneKey{dtype, op, body, log2n});
        return OMPRT_OK;
    }
    if (cfg->num_teams < 1 || cfg->num_teams > 65535 || !valid_threads(cfg->threads_per_team) ||
        (cfg->vec_bytes != 8 && cfg->vec_bytes != 16) ||
        !(cfg->unroll == 1 || cfg->unroll == 2 || cfg->unroll == 4 || cfg->unroll == 8))
        return fail(OMPRT_ERR_INVALID, "tuned configuration must be fully specified and valid");
    g_tune[TuneKey{dtype, op, body, log2n}] =
        LaunchCfg{cfg->num_teams, cfg->threads_per_team, cfg->vec_bytes, cfg->unroll};
    return OMPRT_OK;
}

// ---------------------------------------------------------------- C ABI: runtime

extern "C" omprt_status omprt_workspace_reserve(void* hip_stream, int32_t max_teams,
                                                int32_t max_counters) {
    if (max_teams < 1 || max_teams > 65535)
        return fail(OMPRT_ERR_INVALID, "max_teams %d outside 1..65535", max_teams);
    if (max_counters < 0) return fail(OMPRT_ERR_INVALID, "max_counters < 0");
    Workspace* ws = nullptr;
    return workspace_get(static_cast<hipStream_t>(hip_stream), max_teams, &ws);
}

extern "C" omprt_status omprt_workspace_reset(void* hip_stream) {
    int dev = 0;
    OMPRT_HIP(hipGetDevice(&dev));
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (omprt_status st = array_reset(dev, stream)) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws.find({dev, stream});
    if (it == g_ws.end() || !it->second.base) return OMPRT_OK;
    // counter and flag back to 0; the epoch moves on (stale slot tags stay stale)
    OMPRT_HIP(hipMemsetAsync(it->second.base, 0, 128, stream));
    OMPRT_HIP(hipMemsetAsync(it->second.status(), 0, 4, stream));
    return OMPRT_OK;
}

extern "C" omprt_status omprt_workspace_status(void* hip_stream, int32_t* h_status) {
    if (!h_status) return fail(OMPRT_ERR_INVALID, "status pointer is NULL");
    *h_status = 0;
    int dev = 0;
    OMPRT_HIP(hipGetDevice(&dev));
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    uint32_t* st = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_ws.find({dev, stream});
        if (it != g_ws.end() && it->second.base) st = it->second.status();
    }
    uint32_t v = 0, vb = 0, va = 0;
    OMPRT_HIP(hipStreamSynchronize(stream));
    if (st) OMPRT_HIP(hipMemcpy(&v, st, 4, hipMemcpyDeviceToHost));
    if (uint32_t* bst = batched_status_word(dev, stream))
        OMPRT_HIP(hipMemcpy(&vb, bst, 4, hipMemcpyDeviceToHost));
    if (uint32_t* ast = array_status_word(dev, stream))
        OMPRT_HIP(hipMemcpy(&va, ast, 4, hipMemcpyDeviceToHost));
    *h_status = (int32_t)(v | vb | va);
    return OMPRT_OK;
}

extern "C" const char* omprt_last_error(void) { return t_err.c_str(); }

extern "C" const char* omprt_version(void) { return "omprt 0.1 (gfx950)"; }

extern "C" omprt_status omprt_finalize(void) {
    int dev = 0;
    OMPRT_HIP(hipGetDevice(&dev));
    OMPRT_HIP(hipDeviceSynchronize());
    batched_finalize();
    array_finalize();
    queue_finalize();
    histogram_finalize();
    mlp_finalize();
    udr_finalize();
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_ws) {
        if (!kv.second.base) continue;
        (void)hipSetDevice(kv.first.first);
        (void)hipFree(kv.second.base);
    }
    g_ws.clear();
    g_ws_generation.fetch_add(1, std::memory_order_acq_rel);
    free_retired();
    OMPRT_HIP(hipSetDevice(dev));
    return OMPRT_OK;
}
