// queue.hip -- dynamic and guided worksharing: each distribute block of a
// team is handed out as a queue of chunks that threads take as they ask.
//
// Which thread runs a chunk is not defined for these schedules; the chunks
// themselves are: dynamic chunks are c iterations (the last one shorter),
// guided chunks take ceil(r / P) of the r iterations left, at least c and
// at most r (c = 0 means 1).  Both are therefore a fixed sequence of chunks
// per block size, and the queue hands out chunk numbers: one 64-bit word of
// team-shared memory (LDS) per team, reset at the start of every distribute
// block.  Threads ask a wave at a time: the wave's first active lane takes
// tickets for every active lane with one LDS atomic add and the lanes take
// them in lane order, so the lanes of a wave run neighbouring chunks.
// Dynamic chunk t is [t*c, t*c + c); guided chunk bounds come from a table
// the host computes once per (block size, P, c) and keeps on the device (a
// wave-wide compare-and-swap loop that walks the guided rule per lane costs
// more than the body it schedules).
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "axpy.h"
#include "device.h"
#include "runtime.h"

namespace omprt {

enum { KIND_DYNAMIC = 1, KIND_GUIDED = 2 };

struct QueueCfg {
    int kind;                 // KIND_DYNAMIC or KIND_GUIDED
    int64_t P;                // logical threads of the team
    int64_t cmin;             // chunk size (>= 1)
    int tickets;              // chunks a thread takes per request (>= 1)
    const int64_t* tab[2];    // guided: chunk bounds for block sizes tab_m[0], tab_m[1]
    int64_t tab_m[2];
    int64_t tab_n[2];         // chunks in each table
};

__device__ __forceinline__ uint32_t read_lane(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}
__device__ __forceinline__ uint64_t read_lane64(uint64_t v, int lane) {
    return ((uint64_t)read_lane((uint32_t)(v >> 32), lane) << 32) | read_lane((uint32_t)v, lane);
}

// One request of the calling lane; every active lane of the wave makes it
// together.  On true, the lane's chunks are numbers first + j * stride for
// j < tickets (those at or past nchunks are empty); false: the queue is
// exhausted for this lane.
struct Grab {
    int64_t first, stride;
};
__device__ __forceinline__ bool queue_next(uint64_t* q, int64_t nchunks, int tickets, Grab& g) {
    const uint64_t mask = __ballot(1);
    const int lane = (int)__lane_id();
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    const int cnt = __popcll(mask);
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint64_t base = 0;
    if (lane == leader) base = atomicAdd((unsigned long long*)q, (unsigned long long)cnt * tickets);
    base = read_lane64(base, leader);
    g.first = (int64_t)base + rank;
    g.stride = cnt;
    return g.first < nchunks;
}

// The queue of one block of m iterations: number of chunks, and the bounds
// of chunk t (t < chunks).
struct BlockQueue {
    int64_t m, nchunks;
    const int64_t* tab;   // guided bounds, nchunks + 1 entries
    int64_t c;
    __device__ __forceinline__ BlockQueue(const QueueCfg& qc, int64_t m_) : m(m_), c(qc.cmin) {
        if (qc.kind == KIND_DYNAMIC) {
            tab = nullptr;
            nchunks = (m + c - 1) / c;
        } else {
            const int w = m == qc.tab_m[0] ? 0 : 1;
            tab = qc.tab[w];
            nchunks = qc.tab_n[w];
        }
    }
    __device__ __forceinline__ Range chunk(int64_t t) const {
        if (tab) return Range{tab[t], tab[t + 1]};
        const int64_t lo = t * c;
        return Range{lo, lo + c < m ? lo + c : m};
    }
};

// ---------------------------------------------------------------- iteration map

// owner[i] = team * P + thread of the thread that ran iteration i,
// count[i] += 1, start[i] = first iteration of i's chunk.
__global__ __launch_bounds__(1024) void queue_map_kernel(QueueCfg qc, int64_t n, int64_t dc,
                                                         int32_t* __restrict__ owner,
                                                         uint32_t* __restrict__ count,
                                                         int64_t* __restrict__ start) {
    __shared__ uint64_t queue;
    const int64_t T = gridDim.x, k = blockIdx.x;
    const int t = threadIdx.x;
    const int32_t id = (int32_t)(k * qc.P + t);
    const int64_t nb = team_nblocks(n, T, dc, k);
    for (int64_t b = 0; b < nb; ++b) {
        const Range blk = team_block(n, T, dc, k, b);
        const int64_t m = blk.hi - blk.lo;
        if (t == 0) queue = 0;
        __syncthreads();
        if (t < qc.P) {
            const BlockQueue bq(qc, m);
            Grab g;
            while (queue_next(&queue, bq.nchunks, qc.tickets, g)) {
                for (int j = 0; j < qc.tickets; ++j) {
                    const int64_t tk = g.first + (int64_t)j * g.stride;
                    if (tk >= bq.nchunks) break;
                    const Range ch = bq.chunk(tk);
                    for (int64_t i = ch.lo; i < ch.hi; ++i) {
                        owner[blk.lo + i] = id;
                        atomicAdd(count + blk.lo + i, 1u);
                        start[blk.lo + i] = blk.lo + ch.lo;
                    }
                }
            }
        }
        __syncthreads();   // every thread is done with this block's queue
    }
}

// ---------------------------------------------------------------- AXPY + sum

// ONE: dynamic chunks of one iteration (a separate instantiation, so that
// the register-hungry run code of the other schedules does not cut its
// occupancy: this path is bound by memory latency).  MODE: when a whole
// wave takes tickets and every lane's chunk of a round exists, the wave's
// chunks (neighbouring chunk numbers, so side by side in memory) run
// through a per-wave LDS buffer of 16 KiB (lines.h) instead of lane by lane:
// each lane's run a line per pass (MODE 1: the lines of a wave in rotated
// order, line_rot, for dynamic chunks, whose runs sit a multiple of 4 KiB
// apart for power-of-two chunks; MODE 3: in increasing order, for guided
// chunks, which rotating measured slower), or the union of the wave's runs
// (MODE 2, for dynamic chunks of 16 to kUnionRun iterations).
template <bool ONE, int MODE>
__global__ __launch_bounds__(512) void queue_axpy_kernel(QueueCfg qc, float a,
                                                          const float* __restrict__ x,
                                                          float* __restrict__ y,
                                                          float* __restrict__ sum, int64_t n,
                                                          int64_t dc, CrossTeam ct) {
    using R = Red<DT_F32, OP_SUM>;
    extern __shared__ f32x4 stage[];
    __shared__ uint64_t queue;
    __shared__ ff_t lds_slots[kMaxWaves];
    __shared__ int s_last;
    const int64_t T = gridDim.x, k = blockIdx.x;
    const int t = threadIdx.x;
    const uint32_t epoch = T > 1 ? read_epoch(ct.epoch) : 0u;
    ff_t acc = R::identity();
    const int64_t nb = team_nblocks(n, T, dc, k);
    for (int64_t b = 0; b < nb; ++b) {
        const Range blk = team_block(n, T, dc, k, b);
        const int64_t m = blk.hi - blk.lo;
        if (t == 0) queue = 0;
        __syncthreads();
        if (t < qc.P) {
            const BlockQueue bq(qc, m);
            Grab g;
            const float* xb = x + blk.lo;
            float* yb = y + blk.lo;
            while (queue_next(&queue, bq.nchunks, qc.tickets, g)) {
                if (ONE) {
                    // one-iteration chunks: the lanes of a wave hold neighbouring
                    // iterations; the tickets' loads issue together
                    constexpr int K = 8;
                    float xx[K], yy[K];
                    bool ok[K];
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const int64_t i = g.first + (int64_t)j * g.stride;
                        ok[j] = j < qc.tickets && i < m;
                        const int64_t ii = ok[j] ? i : 0;
                        xx[j] = __builtin_nontemporal_load(xb + ii);
                        yy[j] = __builtin_nontemporal_load(yb + ii);
                    }
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        if (!ok[j]) continue;
                        const int64_t i = g.first + (int64_t)j * g.stride;
                        const float r = __builtin_fmaf(a, xx[j], yy[j]);
                        __builtin_nontemporal_store(r, yb + i);
                        comp_add(acc, r);
                    }
                } else {
                    for (int j = 0; j < qc.tickets; ++j) {
                        const int64_t tk = g.first + (int64_t)j * g.stride;
                        if (MODE && g.stride == kWave &&
                            read_lane64((uint64_t)tk, kWave - 1) < (uint64_t)bq.nchunks) {
                            // the whole wave holds chunks this round (chunk
                            // numbers grow with the lane)
                            f32x4* xs = stage + (size_t)(t / kWave) * (2 * kStageSlots);
                            const Range ch = bq.chunk(tk);
                            if (MODE == 2)
                                axpy_run_union(a, xb, yb, ch.lo, ch.hi, xs, xs + kStageSlots, acc);
                            else
                                axpy_run_lines<MODE == 1>(a, xb, yb, ch.lo, ch.hi, xs,
                                                          xs + kStageSlots, acc);
                            continue;
                        }
                        if (tk >= bq.nchunks) break;
                        const Range ch = bq.chunk(tk);
                        if (ch.hi - ch.lo > 16 || !axpy_short_run(a, xb, yb, ch.lo, ch.hi, acc))
                            axpy_range(a, xb, yb, ch.lo, ch.hi, acc);
                    }
                }
            }
        }
        __syncthreads();
    }
    axpy_finish_sum(acc, sum, ct, epoch, lds_slots, &s_last);
}

// ---------------------------------------------------------------- host side

// Guided chunk bounds of one block of m iterations (nchunks + 1 entries).
static std::vector<int64_t> guided_bounds(int64_t m, int64_t P, int64_t cmin) {
    std::vector<int64_t> b{0};
    int64_t s = 0;
    while (s < m) {
        const int64_t r = m - s;
        int64_t size = (r + P - 1) / P;
        if (size < cmin) size = cmin;
        if (size > r) size = r;
        s += size;
        b.push_back(s);
    }
    return b;
}

// Device copies of guided tables, per (device, block size, P, c); read-only
// once uploaded, kept until omprt_finalize.
struct TableKey {
    int dev;
    int64_t m, P, c;
    bool operator<(const TableKey& o) const {
        return std::tie(dev, m, P, c) < std::tie(o.dev, o.m, o.P, o.c);
    }
};
struct DevTable {
    int64_t* ptr = nullptr;
    int64_t nchunks = 0;
};
static std::mutex g_qmu;
static std::map<TableKey, DevTable> g_tables;
constexpr size_t kMaxTables = 1024;

static omprt_status guided_table(hipStream_t stream, int64_t m, int64_t P, int64_t cmin,
                                 DevTable* out) {
    int dev = 0;
    OMPRT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_qmu);
    const TableKey key{dev, m, P, cmin};
    auto it = g_tables.find(key);
    if (it != g_tables.end()) {
        *out = it->second;
        return OMPRT_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    OMPRT_HIP(hipStreamIsCapturing(stream, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return fail(OMPRT_ERR_INVALID,
                    "stream is being captured and the guided table for this block size is not "
                    "built yet: make the same call once before capturing");
    if (g_tables.size() >= kMaxTables) {
        // many distinct block sizes: start a new cache (captured graphs may still name
        // the old tables, so they wait for omprt_finalize)
        for (auto& kv : g_tables) retire_device_memory(kv.first.dev, kv.second.ptr);
        g_tables.clear();
    }
    const std::vector<int64_t> b = guided_bounds(m, P, cmin);
    DevTable t;
    t.nchunks = (int64_t)b.size() - 1;
    if (hipMalloc(&t.ptr, b.size() * sizeof(int64_t)) != hipSuccess)
        return fail(OMPRT_ERR_NOMEM, "guided table of %zu entries", b.size());
    // synchronous: the table is complete before any stream can use it
    OMPRT_HIP(hipMemcpy(t.ptr, b.data(), b.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    g_tables[key] = t;
    *out = t;
    return OMPRT_OK;
}

void queue_finalize() {
    std::lock_guard<std::mutex> lk(g_qmu);
    for (auto& kv : g_tables) {
        (void)hipSetDevice(kv.first.dev);
        (void)hipFree(kv.second.ptr);
    }
    g_tables.clear();
}

// Block sizes of a launch's non-empty distribute blocks (at most two).
static int block_sizes(int64_t n, int64_t T, int64_t dc, int64_t out[2]) {
    int k = 0;
    auto add = [&](int64_t m) {
        if (m > 0 && (k == 0 || out[0] != m)) out[k++] = m;
    };
    if (dc == 0) {
        add(n / T + (n % T ? 1 : 0));   // the first n % T teams
        add(n / T);
    } else {
        if (n >= dc) add(dc);
        add(n % dc);
    }
    return k;
}

static omprt_status make_cfg(hipStream_t stream, int kind, int64_t n, int64_t T, int P,
                             int64_t dc, int64_t c, int tickets, QueueCfg* out) {
    QueueCfg qc{};
    qc.kind = kind;
    qc.P = P;
    qc.cmin = c > 0 ? c : 1;
    qc.tickets = tickets;
    if (kind == KIND_GUIDED) {
        int64_t ms[2] = {0, 0};
        const int k = block_sizes(n, T, dc, ms);
        for (int i = 0; i < k; ++i) {
            DevTable t;
            if (omprt_status st = guided_table(stream, ms[i], P, qc.cmin, &t)) return st;
            qc.tab[i] = t.ptr;
            qc.tab_m[i] = ms[i];
            qc.tab_n[i] = t.nchunks;
        }
        for (int i = k; i < 2; ++i) {   // unused slot: a copy of the first
            qc.tab[i] = qc.tab[0];
            qc.tab_m[i] = qc.tab_m[0];
            qc.tab_n[i] = qc.tab_n[0];
        }
    }
    *out = qc;
    return OMPRT_OK;
}

}  // namespace omprt

using namespace omprt;

static omprt_status check_queue(const omprt_sched* s, int32_t kind) {
    if (kind != KIND_DYNAMIC && kind != KIND_GUIDED)
        return fail(OMPRT_ERR_INVALID, "schedule kind %d (1 dynamic, 2 guided)", kind);
    return check_sched(s, false);
}

extern "C" omprt_status omprt_queue_map(const omprt_sched* s, int32_t kind, int32_t tickets,
                                        int32_t* d_owner, uint32_t* d_count, int64_t* d_start,
                                        void* hip_stream) {
    if (omprt_status st = check_queue(s, kind)) return st;
    if (tickets < 1 || tickets > 64)
        return fail(OMPRT_ERR_INVALID, "tickets %d outside 1..64", tickets);
    if ((int64_t)s->num_teams * s->threads_per_team > INT32_MAX)
        return fail(OMPRT_ERR_INVALID, "num_teams * threads_per_team exceeds int32 owner ids");
    if (s->n == 0) return OMPRT_OK;
    if (!d_owner || !d_count || !d_start) return fail(OMPRT_ERR_INVALID, "owner/count/start is NULL");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    QueueCfg qc;
    if (omprt_status st = make_cfg(stream, kind, s->n, s->num_teams, s->threads_per_team,
                                   s->dist_chunk, s->chunk, tickets, &qc))
        return st;
    const int block = (s->threads_per_team + kWave - 1) / kWave * kWave;
    hipLaunchKernelGGL(queue_map_kernel, dim3(s->num_teams), dim3(block), 0, stream, qc, s->n,
                       s->dist_chunk, d_owner, d_count, d_start);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "queue map launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}

extern "C" omprt_status omprt_axpy_sum_queue(float a, const float* d_x, float* d_y, float* d_sum,
                                             const omprt_sched* s, int32_t kind,
                                             void* hip_stream) {
    if (kind != KIND_DYNAMIC && kind != KIND_GUIDED)
        return fail(OMPRT_ERR_INVALID, "schedule kind %d (1 dynamic, 2 guided)", kind);
    if (omprt_status st = check_sched(s, true)) return st;
    if (!d_sum) return fail(OMPRT_ERR_INVALID, "sum is NULL");
    if (s->n > 0 && (!d_x || !d_y)) return fail(OMPRT_ERR_INVALID, "x/y is NULL with n > 0");
    if ((reinterpret_cast<uintptr_t>(d_x) | reinterpret_cast<uintptr_t>(d_y) |
         reinterpret_cast<uintptr_t>(d_sum)) & 3)
        return fail(OMPRT_ERR_INVALID, "x/y/sum not 4-byte aligned");
    if (s->n > 0) {
        const char* xb = reinterpret_cast<const char*>(d_x);
        const char* yb = reinterpret_cast<const char*>(d_y);
        if (xb < yb + s->n * 4 && yb < xb + s->n * 4)
            return fail(OMPRT_ERR_INVALID, "x and y overlap");
    }
    const int teams = s->num_teams ? s->num_teams : device_cus();
    if (teams > 65535)
        return fail(OMPRT_ERR_INVALID, "num_teams %d above 65535 (cross-team slot limit)", teams);
    // default team size: 512 threads for dynamic chunks under 16 iterations
    // (more lanes asking at once), else 256 (for guided also fewer, longer
    // chunks): 2^26 fp32 on gfx950, dynamic 1 4.50 against 2.65 TB/s with
    // 256, dynamic 64 5.16 against 5.11, guided 1 4.07 against 3.39, guided
    // 64 4.31 against 3.75
    const int threads = s->threads_per_team ? s->threads_per_team
                        : (kind == KIND_DYNAMIC && s->chunk < 16) ? 512
                                                                   : 256;
    if (threads > 512)
        return fail(OMPRT_ERR_INVALID, "threads_per_team %d above 512 for this body", threads);
    if (s->n == 0) return OMPRT_OK;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    Workspace* ws = nullptr;
    if (omprt_status st = workspace_get(stream, teams, &ws)) return st;
    const CrossTeamArgs ca = ws->cross();
    const CrossTeam ct{static_cast<uint64_t*>(ca.slots), ca.counter, ca.epoch, ca.status};
    // one-iteration dynamic chunks: eight per request, so that eight loads of
    // each stream are in flight per lane and a wave's LDS atomic covers 512
    // iterations (2^26 fp32, default launch: 4.45 TB/s with four, 4.98 with
    // eight; 256-thread teams 2.66 against 3.98)
    const int tickets = (kind == KIND_DYNAMIC && s->chunk <= 1) ? 8 : 1;
    QueueCfg qc;
    if (omprt_status st = make_cfg(stream, kind, s->n, teams, threads, s->dist_chunk, s->chunk,
                                   tickets, &qc))
        return st;
    const int block = (threads + kWave - 1) / kWave * kWave;
    // lines for chunks of at least 64 iterations (dynamic) and for guided
    // chunks (they start at m / P iterations), teams of whole waves, x and y
    // co-aligned to 16 bytes; dynamic chunks of 32 to 64 iterations (8 to
    // 31 when the team blocks are off the 32-element grid of y) as the union
    // of the wave's runs, except whole-line chunks of 64.  2^26 fp32, one
    // team of 256 a CU: chunk 32 4.03 -> 5.06 TB/s; blocks off the grid:
    // chunk 16 2.03 -> 3.03, 32 2.66 -> 3.32, 64 3.04 -> 3.87; longer chunks
    // (100, 128) and chunk 16 on the grid ran slower through the union
    // (four waves a CU hide less of its per-lane LDS work than the static
    // schedules' eight).  Off the grid, chunks 8 and 12 (one team of 512 a
    // CU): 1.84 -> 2.90 and 2.53 -> 3.87 TB/s through the union; chunks 2 and
    // 4 ran slower through it (2.23 -> 0.97, 2.86 -> 1.92), 7 alike.
    const bool co = ((reinterpret_cast<uintptr_t>(d_x) ^ reinterpret_cast<uintptr_t>(d_y)) & 15) == 0;
    const bool waves = threads % kWave == 0;
    const bool on_grid = (reinterpret_cast<uintptr_t>(d_y) & (kLineBytes - 1)) == 0 &&
                         (s->dist_chunk ? s->dist_chunk % 32 == 0
                                        : s->n % teams == 0 && (s->n / teams) % 32 == 0);
    const int64_t c = qc.cmin;
    const bool union_runs = kind == KIND_DYNAMIC &&
                            ((c >= 32 && c <= 64 && !(on_grid && c == 64)) ||
                             (c >= 8 && c < 32 && !on_grid));
    const bool lines = waves && co && (kind == KIND_GUIDED || qc.cmin >= 64);
    hipError_t e = hipSuccess;
    auto launch_staged = [&](auto kernel) {
        const size_t lds = (size_t)(threads / kWave) * 2 * kStageSlots * 16;
        if (lds > 64 * 1024)   // past the default dynamic LDS limit: ask for it
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e == hipSuccess)
            hipLaunchKernelGGL(kernel, dim3(teams), dim3(block), lds, stream, qc, a, d_x, d_y,
                               d_sum, s->n, s->dist_chunk, ct);
    };
    if (kind == KIND_DYNAMIC && qc.cmin == 1) {
        hipLaunchKernelGGL((queue_axpy_kernel<true, 0>), dim3(teams), dim3(block), 0, stream,
                           qc, a, d_x, d_y, d_sum, s->n, s->dist_chunk, ct);
    } else if (waves && co && union_runs) {
        launch_staged(queue_axpy_kernel<false, 2>);
    } else if (lines && kind == KIND_DYNAMIC) {
        launch_staged(queue_axpy_kernel<false, 1>);
    } else if (lines) {
        launch_staged(queue_axpy_kernel<false, 3>);
    } else {
        hipLaunchKernelGGL((queue_axpy_kernel<false, 0>), dim3(teams), dim3(block), 0, stream,
                           qc, a, d_x, d_y, d_sum, s->n, s->dist_chunk, ct);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(OMPRT_ERR_DEVICE, "queue axpy launch: %s", hipGetErrorString(e));
    return OMPRT_OK;
}

extern "C" omprt_status omprt_queue_chunk(int32_t kind, int64_t m, int32_t threads, int64_t chunk,
                                          int64_t j, int64_t* lb, int64_t* ub) {
    if (kind != KIND_DYNAMIC && kind != KIND_GUIDED)
        return fail(OMPRT_ERR_INVALID, "schedule kind %d (1 dynamic, 2 guided)", kind);
    if (m < 0 || m > ((int64_t)1 << 50) || threads < 1 || threads > 1024 || chunk < 0 || j < 0)
        return fail(OMPRT_ERR_INVALID, "bad queue arguments");
    if (!lb || !ub) return fail(OMPRT_ERR_INVALID, "NULL output");
    const int64_t c = chunk > 0 ? chunk : 1;
    if (kind == KIND_DYNAMIC) {
        const int64_t lo = j < (m + c - 1) / c ? j * c : m;
        *lb = lo;
        *ub = lo + c < m ? lo + c : m;
        return OMPRT_OK;
    }
    // the same bounds the guided kernels' tables hold
    const std::vector<int64_t> b = guided_bounds(m, threads, c);
    const int64_t nch = (int64_t)b.size() - 1;
    *lb = j < nch ? b[j] : m;
    *ub = j < nch ? b[j + 1] : m;
    return OMPRT_OK;
}
