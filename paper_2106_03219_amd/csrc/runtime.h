// runtime.h -- internal host-runtime interfaces shared by the C-ABI
// translation units: error reporting, workspaces, configuration resolution.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/omprt.h"

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

// Per (device, stream) workspace of the plain kernels: one cross-team
// counter (zeroed once at allocation, self-resetting afterwards) and the
// cross-team partial slots.
struct Workspace {
    void* base = nullptr;
    int32_t capacity = 0;   // slots
    uint32_t* counter() const { return static_cast<uint32_t*>(base); }
    int32_t* flag() const { return static_cast<int32_t*>(base) + 16; }
    void* slots() const { return static_cast<char*>(base) + 256; }
};

// Workspace of `stream` with room for `teams` slots, allocated or grown
// here (never while the stream is being captured).
omprt_status workspace_get(hipStream_t stream, int32_t teams, Workspace** out);

struct LaunchCfg {
    int teams, threads, vec, unroll;
};
enum ConfigSource { kSrcExplicit = 0, kSrcModel = 1, kSrcTuned = 2, kSrcHeuristic = 3 };

// Explicit fields of cfg win; the rest come from the learned model, else the
// tuned cache, else the heuristic.  body: 0 reduction, 1 AXPY.
omprt_status resolve_config(int64_t n, int dtype, int op, int body, int64_t chunk,
                            const omprt_config* cfg, LaunchCfg* out, int* source);

// Learned picker (model.hip): true and *out filled when a model is loaded
// and confident for these features.
bool model_pick(const float* features16, int body, int64_t n, LaunchCfg* out);
void model_features(int64_t n, int dtype, int op, int body, int64_t chunk, float* f16);

}  // namespace omprt
