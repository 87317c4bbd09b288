// runtime.h -- internal host-runtime interfaces shared by the C-ABI
// translation units: error reporting, workspaces, configuration resolution.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/omprt.h"
#include "launch.h"
#include "ops.h"

namespace omprt {

// Record a message for omprt_last_error() and return st.
omprt_status fail(omprt_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
omprt_status ok();

#define OMPRT_HIP(call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::omprt::fail(OMPRT_ERR_DEVICE, "%s failed: %s", #call,               \
                                 hipGetErrorString(e_));                                 \
    } while (0)

constexpr int DT_COUNT_ABI = 5;   // OMPRT_I32 .. OMPRT_BF16

int dtype_bytes(int dtype);         // storage bytes of an input element
int out_bytes(int dtype, int op);   // bytes of x

// Per (device, stream) workspace of the plain kernels: a 256-byte header
// (election counter, launch epoch, status bits; zeroed once at allocation,
// self-maintaining afterwards) followed by the tagged cross-team slots.
struct Workspace {
    void* base = nullptr;
    int32_t capacity = 0;   // slots
    uint32_t* counter() const { return static_cast<uint32_t*>(base); }
    uint32_t* epoch() const { return static_cast<uint32_t*>(base) + 32; }
    uint32_t* status() const { return static_cast<uint32_t*>(base) + 48; }
    void* slots() const { return static_cast<char*>(base) + 256; }
    CrossTeamArgs cross() const { return CrossTeamArgs{slots(), counter(), epoch(), status()}; }
};

// Device memory a caller's captured graph may still name is never freed while
// the library is in use: a buffer that a larger one supersedes waits on this
// list (no synchronisation needed) until omprt_finalize frees it.
void retire_device_memory(int dev, void* p);

// Workspace of `stream` with room for `teams` slots, allocated or grown
// here (never while the stream is being captured).
omprt_status workspace_get(hipStream_t stream, int32_t teams, Workspace** out);

struct LaunchCfg {
    int teams, threads, vec, unroll;
};
enum ConfigSource { kSrcExplicit = 0, kSrcModel = 1, kSrcTuned = 2, kSrcHeuristic = 3 };

// Explicit fields of cfg win; the rest come from the learned model, else the
// tuned cache, else the heuristic.  body: 0 reduction, 1 AXPY, 2 the
// AXPY-then-sum region (the AXPY's model features and tuned entries, a
// heuristic of its own).
omprt_status resolve_config(int64_t n, int dtype, int op, int body, int64_t chunk,
                            const omprt_config* cfg, LaunchCfg* out, int* source);

// Validate a schedule (allow_auto: num_teams / threads_per_team may be 0).
omprt_status check_sched(const omprt_sched* s, bool allow_auto);

// Compute units of the current device (256 if it cannot be queried).
int device_cus();

// Batched plans (batched.hip): free everything; status word of a stream's plan.
void batched_finalize();
uint32_t* batched_status_word(int dev, hipStream_t stream);

// MLP kernels (mlp.hip): free the scratch buffers.
void mlp_finalize();

// Histograms (histogram.hip): free the pools.
void histogram_finalize();

// User-defined reductions (udr.hip): unload the loaded modules.
void udr_finalize();

// Dynamic / guided worksharing (queue.hip): free the guided tables.
void queue_finalize();

// Array-section reductions (array.hip): free everything; status word of a
// stream's workspace; re-zero its counters and status.
void array_finalize();
uint32_t* array_status_word(int dev, hipStream_t stream);
omprt_status array_reset(int dev, hipStream_t stream);

// Learned picker (model.hip): true and *out filled when a model is loaded
// and confident for these features.
bool model_pick(int64_t n, int dtype, int op, int body, int64_t chunk, LaunchCfg* out);
void model_features(int64_t n, int dtype, int op, int body, int64_t chunk, float* f16);

}  // namespace omprt
