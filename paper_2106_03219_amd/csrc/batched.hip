// batched.hip -- many independent reductions in one persistent launch.
//
// A plan splits every segment into tiles of a fixed byte size (a segment
// shorter than one tile is one tile).  A grid of one device-wide wave of
// workgroups takes tiles either by an atomic ticket (the wrap-around
// increment again, with bound ntiles + G - 1, so the ticket returns to 0
// when every workgroup has drawn its final, out-of-range ticket) or
// round-robin.  Each tile is streamed and team-reduced exactly like a plain
// reduction's team block; a multi-tile segment's tile partials go to fixed
// slots and the segment's own wrap-increment counter (bound tiles - 1)
// elects the tile that finishes last to combine them in tile order and
// write x.  Slots are tagged with the launch epoch like the plain kernels'
// (device.h); a launch-wide wrap-increment over finished segments elects the
// workgroup that advances the epoch.  Results do not depend on which
// workgroup ran which tile.  The launch is captured once into a HIP graph
// and replayed: counters, ticket and epoch maintain themselves, so replays
// need no memset.
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "device.h"
#include "launch.h"
#include "runtime.h"
#include "stream.h"

namespace omprt {

struct SegDesc {
    const void* in;
    void* x;
    int64_t n;
    int32_t dtype, op;
    int32_t first_tile, ntiles;
};

struct TileDesc {
    int64_t lo, hi;
    int32_t seg, pad;
};

// Device state of one plan: tagged slot per tile, election counter per
// segment, tile ticket, finished-segment counter, epoch and status words.
struct BatchState {
    uint64_t* slots;
    uint32_t* seg_counters;
    uint32_t* ticket;
    uint32_t* done;
    uint32_t* epoch;
    uint32_t* status;
    int32_t ntiles;
    int32_t nseg_active;   // segments with at least one tile
};

// Reduce one tile; returns true (team-uniform) if it completed its segment.
template <int DT, int OP, int VB, int U>
__device__ __forceinline__ bool process_tile(const SegDesc& sd, const TileDesc& td, int tile,
                                             const BatchState& bs, uint32_t tag, void* lds_raw,
                                             int* s_last) {
    using R = Red<DT, OP>;
    using Acc = typename R::Acc;
    Acc acc[R::kNA];
#pragma unroll
    for (int i = 0; i < R::kNA; ++i) acc[i] = R::identity();
    stream_range<DT, OP, VB, U>(static_cast<const typename DType<DT>::S*>(sd.in), td.lo, td.hi,
                                acc);
    Acc t = acc[0];
#pragma unroll
    for (int i = 1; i < R::kNA; ++i) t = R::combine(t, acc[i]);
    Acc* lds = static_cast<Acc*>(lds_raw);
    t = team_reduce<R>(t, lds);
    typename R::Out* x = static_cast<typename R::Out*>(sd.x);
    if (sd.ntiles == 1) {
        if (threadIdx.x == 0) x[0] = R::finish(t, x[0]);
        return true;
    }
    if (!publish_and_elect(t, bs.slots + (size_t)tile * kSlotWords, bs.seg_counters + td.seg,
                           (uint32_t)(sd.ntiles - 1), tag, s_last))
        return false;
    const Acc c = combine_slots<R>(bs.slots + (size_t)sd.first_tile * kSlotWords, sd.ntiles, tag,
                                   bs.status, lds);
    if (threadIdx.x == 0) x[0] = R::finish(c, x[0]);
    return true;
}

template <int VB, int U>
__global__ __launch_bounds__(1024) void batched_kernel(const SegDesc* __restrict__ segs,
                                                       const TileDesc* __restrict__ tiles,
                                                       BatchState bs, int32_t use_ticket) {
    __shared__ Pair<double> lds[kMaxWaves];
    __shared__ int s_tile;
    __shared__ int s_last;
    const uint32_t epoch = read_epoch(bs.epoch);
    const uint32_t tag = launch_tag(epoch);
    int32_t next = blockIdx.x;
    for (;;) {
        __syncthreads();   // LDS from the previous tile is no longer read
        int32_t tile;
        if (use_ticket) {
            if (threadIdx.x == 0)
                s_tile = (int)__builtin_amdgcn_atomic_inc32(
                    bs.ticket, (uint32_t)(bs.ntiles + gridDim.x - 1), __ATOMIC_RELAXED, "agent");
            __syncthreads();
            tile = s_tile;
        } else {
            tile = next;
            next += gridDim.x;
        }
        if (tile >= bs.ntiles) break;
        const TileDesc td = tiles[tile];
        const SegDesc sd = segs[td.seg];
        bool seg_done = false;
        switch (sd.dtype * OP_COUNT + sd.op) {
#define OMPRT_CASE(DT, OP)                                                               \
    case DT * OP_COUNT + OP:                                                             \
        seg_done = process_tile<DT, OP, VB, U>(sd, td, tile, bs, tag, lds, &s_last);     \
        break;
            OMPRT_CASE(DT_I32, OP_SUM) OMPRT_CASE(DT_I32, OP_MAX) OMPRT_CASE(DT_I32, OP_MIN)
            OMPRT_CASE(DT_I64, OP_SUM) OMPRT_CASE(DT_I64, OP_MAX) OMPRT_CASE(DT_I64, OP_MIN)
            OMPRT_CASE(DT_F32, OP_SUM) OMPRT_CASE(DT_F32, OP_MAX) OMPRT_CASE(DT_F32, OP_MIN)
            OMPRT_CASE(DT_F64, OP_SUM) OMPRT_CASE(DT_F64, OP_MAX) OMPRT_CASE(DT_F64, OP_MIN)
            OMPRT_CASE(DT_BF16, OP_SUM) OMPRT_CASE(DT_BF16, OP_MAX) OMPRT_CASE(DT_BF16, OP_MIN)
#undef OMPRT_CASE
            default: break;
        }
        // the workgroup that completes the launch's last segment advances the epoch
        if (seg_done && threadIdx.x == 0) {
            const uint32_t e = (uint32_t)(bs.nseg_active - 1);
            if (__builtin_amdgcn_atomic_inc32(bs.done, e, __ATOMIC_RELAXED, "agent") == e)
                advance_epoch(bs.epoch, epoch);
        }
    }
}

using BatchedKernel = void (*)(const SegDesc*, const TileDesc*, BatchState, int32_t);

static BatchedKernel batched_variant(int vec, int unroll) {
    if (vec == 16) {
        switch (unroll) {
            case 1: return batched_kernel<16, 1>;
            case 2: return batched_kernel<16, 2>;
            case 4: return batched_kernel<16, 4>;
            case 8: return batched_kernel<16, 8>;
        }
    } else if (vec == 8) {
        switch (unroll) {
            case 1: return batched_kernel<8, 1>;
            case 2: return batched_kernel<8, 2>;
            case 4: return batched_kernel<8, 4>;
            case 8: return batched_kernel<8, 8>;
        }
    }
    return nullptr;
}

// ---------------------------------------------------------------- plans

struct Plan {
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<omprt_segment> segs;
    omprt_config cfg{};
    void* dmem = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t ntiles = 0;
    uint32_t* status = nullptr;
    // Explicit, never from a destructor: a plan still alive when the process
    // exits is left to the driver (no HIP call runs from static destruction).
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (dmem) (void)hipFree(dmem);
        exec = nullptr;
        graph = nullptr;
        dmem = nullptr;
    }
};

static std::mutex g_bmu;
// one cached plan per (device, stream): a repeat call with the same segment
// list and configuration replays its graph
static std::map<std::pair<int, hipStream_t>, std::unique_ptr<Plan>> g_plans;
// superseded plans: a graph the caller captured around an earlier call may
// still replay their launch, so they live until omprt_finalize
static std::vector<std::unique_ptr<Plan>> g_retired_plans;
static std::map<int, hipStream_t> g_capture_stream;

static bool same_plan(const Plan& p, const omprt_segment* s, int32_t count,
                      const omprt_config& cfg) {
    if ((int32_t)p.segs.size() != count) return false;
    if (memcmp(&p.cfg, &cfg, sizeof cfg) != 0) return false;
    return memcmp(p.segs.data(), s, sizeof(omprt_segment) * (size_t)count) == 0;
}

static omprt_status check_segments(const omprt_segment* s, int32_t count) {
    for (int32_t i = 0; i < count; ++i) {
        const omprt_segment& g = s[i];
        if (g.dtype < 0 || g.dtype >= DT_COUNT_ABI || g.op < 0 || g.op > 2)
            return fail(OMPRT_ERR_UNSUPPORTED, "segment %d: dtype %d / op %d", i, g.dtype, g.op);
        if (g.n < 0 || g.n > ((int64_t)1 << 50))
            return fail(OMPRT_ERR_INVALID, "segment %d: n outside 0..2^50", i);
        if (!g.d_x) return fail(OMPRT_ERR_INVALID, "segment %d: x is NULL", i);
        if (g.n > 0 && !g.d_in) return fail(OMPRT_ERR_INVALID, "segment %d: input is NULL", i);
        if (reinterpret_cast<uintptr_t>(g.d_in) % (uintptr_t)dtype_bytes(g.dtype) ||
            reinterpret_cast<uintptr_t>(g.d_x) % (uintptr_t)out_bytes(g.dtype, g.op))
            return fail(OMPRT_ERR_INVALID, "segment %d: misaligned pointer", i);
    }
    return OMPRT_OK;
}

// Defaults of the batched launch: 1024 threads, 16-byte loads, unroll 4,
// 1 MiB tiles, one workgroup per 1024 threads of device capacity (two a
// CU), ticket.  Over 4096 segments of 10^2..10^7 elements (16 GB) on
// gfx950: 2.34 ms, against 2.54 with 256 threads and 256 KiB tiles, 2.37
// with 1024 threads and 256 KiB, 2.33 with 4 MiB.
static void batched_defaults(const omprt_config* cfg, omprt_config* out, int cus) {
    omprt_config c{};
    if (cfg) c = *cfg;
    if (!c.threads_per_team) c.threads_per_team = 1024;
    if (!c.vec_bytes) c.vec_bytes = 16;
    if (!c.unroll) c.unroll = 4;
    if (!c.tile_kib) c.tile_kib = 1024;
    if (!c.num_teams) c.num_teams = cus * (2048 / c.threads_per_team);
    c.flags &= OMPRT_CFG_STATIC_TILES;
    *out = c;
}

static omprt_status build_plan(Plan& p, hipStream_t user_stream) {
    const int32_t count = (int32_t)p.segs.size();
    const int64_t tile_bytes = (int64_t)p.cfg.tile_kib * 1024;
    std::vector<SegDesc> sd((size_t)count);
    std::vector<TileDesc> td;
    for (int32_t i = 0; i < count; ++i) {
        const omprt_segment& g = p.segs[i];
        const int eb = dtype_bytes(g.dtype);
        const int64_t te = std::max<int64_t>(tile_bytes / eb, 1);
        const int64_t nt = g.n == 0 ? 0 : (g.n - 1) / te + 1;
        if ((int64_t)td.size() + nt > INT32_MAX / 2)
            return fail(OMPRT_ERR_INVALID, "batched plan: too many tiles (raise tile_kib)");
        sd[i] = SegDesc{g.d_in, g.d_x, g.n, g.dtype, g.op, (int32_t)td.size(), (int32_t)nt};
        for (int64_t t = 0; t < nt; ++t)
            td.push_back(TileDesc{t * te, std::min(g.n, (t + 1) * te), i, 0});
    }
    p.ntiles = (int32_t)td.size();
    int32_t active = 0;
    for (const SegDesc& d : sd) active += d.ntiles > 0 ? 1 : 0;
    const size_t seg_b = (sizeof(SegDesc) * (size_t)count + 255) / 256 * 256;
    const size_t tile_b = (sizeof(TileDesc) * td.size() + 255) / 256 * 256;
    const size_t slot_b = ((size_t)kSlotBytes * td.size() + 255) / 256 * 256;
    const size_t ctr_b = ((size_t)(count + 4) * 4 + 255) / 256 * 256;
    if (hipMalloc(&p.dmem, seg_b + tile_b + slot_b + ctr_b) != hipSuccess)
        return fail(OMPRT_ERR_NOMEM, "batched plan allocation failed");
    char* base = static_cast<char*>(p.dmem);
    SegDesc* d_seg = reinterpret_cast<SegDesc*>(base);
    TileDesc* d_tile = reinterpret_cast<TileDesc*>(base + seg_b);
    uint32_t* d_ctr = reinterpret_cast<uint32_t*>(base + seg_b + tile_b + slot_b);
    BatchState bs{reinterpret_cast<uint64_t*>(base + seg_b + tile_b), d_ctr, d_ctr + count,
                  d_ctr + count + 1, d_ctr + count + 2, d_ctr + count + 3, p.ntiles, active};
    if (count) OMPRT_HIP(hipMemcpy(d_seg, sd.data(), sizeof(SegDesc) * sd.size(), hipMemcpyHostToDevice));
    if (!td.empty())
        OMPRT_HIP(hipMemcpy(d_tile, td.data(), sizeof(TileDesc) * td.size(), hipMemcpyHostToDevice));
    // once: zero slots (odd tags never match 0) and every counter
    OMPRT_HIP(hipMemsetAsync(base + seg_b + tile_b, 0, slot_b + ctr_b, user_stream));
    OMPRT_HIP(hipStreamSynchronize(user_stream));
    p.status = bs.status;

    BatchedKernel k = batched_variant(p.cfg.vec_bytes, p.cfg.unroll);
    if (!k) return fail(OMPRT_ERR_INVALID, "no batched kernel for vec %d unroll %d",
                        p.cfg.vec_bytes, p.cfg.unroll);
    hipStream_t cs = g_capture_stream[p.device];
    if (!cs) {
        OMPRT_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        g_capture_stream[p.device] = cs;
    }
    const int32_t use_ticket = (p.cfg.flags & OMPRT_CFG_STATIC_TILES) ? 0 : 1;
    const int grid = std::max(1, std::min<int>(p.cfg.num_teams, std::max<int32_t>(p.ntiles, 1)));
    OMPRT_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(k, dim3(grid), dim3(p.cfg.threads_per_team), 0, cs, d_seg, d_tile, bs,
                       use_ticket);
    const hipError_t le = hipGetLastError();
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(cs, &g);
    if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(OMPRT_ERR_DEVICE, "batched capture failed: %s / %s", hipGetErrorString(le),
                    hipGetErrorString(ce));
    }
    p.graph = g;
    OMPRT_HIP(hipGraphInstantiate(&p.exec, g, nullptr, nullptr, 0));
    return OMPRT_OK;
}

void batched_finalize() {
    std::lock_guard<std::mutex> lk(g_bmu);
    for (auto& kv : g_plans)
        if (kv.second) {
            (void)hipSetDevice(kv.second->device);
            kv.second->release();
        }
    for (auto& p : g_retired_plans) {
        (void)hipSetDevice(p->device);
        p->release();
    }
    g_plans.clear();
    g_retired_plans.clear();
    for (auto& kv : g_capture_stream)
        if (kv.second) (void)hipStreamDestroy(kv.second);
    g_capture_stream.clear();
}

}  // namespace omprt

using namespace omprt;

extern "C" omprt_status omprt_reduce_batched(const omprt_segment* h_segs, int32_t count,
                                             const omprt_config* cfg, void* hip_stream) {
    if (count < 0) return fail(OMPRT_ERR_INVALID, "count < 0");
    if (count > 0 && !h_segs) return fail(OMPRT_ERR_INVALID, "segments pointer is NULL");
    if (count == 0) return OMPRT_OK;
    if (omprt_status st = check_segments(h_segs, count)) return st;
    LaunchCfg dummy;
    if (omprt_status st = resolve_config(1, OMPRT_F32, OMPRT_SUM, 0, -1, cfg, &dummy, nullptr))
        return st;   // field validation only
    int dev = 0, cus = 0;
    OMPRT_HIP(hipGetDevice(&dev));
    OMPRT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    omprt_config c;
    batched_defaults(cfg, &c, cus);
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::mutex> lk(g_bmu);
    std::unique_ptr<Plan>& slot = g_plans[{dev, stream}];
    if (!slot || !same_plan(*slot, h_segs, count, c)) {
        hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
        OMPRT_HIP(hipStreamIsCapturing(stream, &cst));
        if (cst != hipStreamCaptureStatusNone)
            return fail(OMPRT_ERR_INVALID, "omprt_reduce_batched builds its plan outside capture");
        if (slot) g_retired_plans.push_back(std::move(slot));   // replays may still run
        std::unique_ptr<Plan> p(new Plan());
        p->device = dev;
        p->stream = stream;
        p->segs.assign(h_segs, h_segs + count);
        p->cfg = c;
        if (omprt_status st = build_plan(*p, stream)) {
            p->release();
            return st;
        }
        slot = std::move(p);
    }
    if (slot->ntiles == 0) return OMPRT_OK;
    OMPRT_HIP(hipGraphLaunch(slot->exec, stream));
    return OMPRT_OK;
}

extern "C" omprt_status omprt_reduce_each(const omprt_segment* h_segs, int32_t count,
                                          const omprt_config* cfg, void* hip_stream) {
    if (count < 0) return fail(OMPRT_ERR_INVALID, "count < 0");
    if (count > 0 && !h_segs) return fail(OMPRT_ERR_INVALID, "segments pointer is NULL");
    if (omprt_status st = check_segments(h_segs, count)) return st;
    for (int32_t i = 0; i < count; ++i) {
        const omprt_segment& g = h_segs[i];
        if (omprt_status st = omprt_reduce(g.d_in, g.n, g.dtype, g.op, g.d_x, cfg, hip_stream))
            return st;
    }
    return OMPRT_OK;
}

namespace omprt {
// Status word of the stream's cached batched plan (nullptr if none).
uint32_t* batched_status_word(int dev, hipStream_t stream) {
    std::lock_guard<std::mutex> lk(g_bmu);
    auto it = g_plans.find({dev, stream});
    return (it == g_plans.end() || !it->second) ? nullptr : it->second->status;
}
}  // namespace omprt
