// atomics.hip -- the device runtime's five atomic operations (add, inc,
// max, exchange, cas), applied concurrently by one GPU thread each.
//
// inc keeps the wrap-around definition { v = x; x = x >= e ? 0 : x + 1 }
// and uses the AMDGPU builtin that implements it; the others are the
// compare/capture forms with 32-bit unsigned operands.  All are sequentially
// consistent at agent scope.
#include "device.h"
#include "runtime.h"

namespace omprt {

__global__ __launch_bounds__(256) void atomic_apply_kernel(int op, uint32_t* __restrict__ target,
                                                           int64_t n_targets,
                                                           const uint32_t* __restrict__ index,
                                                           const uint32_t* __restrict__ e,
                                                           const uint32_t* __restrict__ d,
                                                           uint32_t* __restrict__ old, int64_t n,
                                                           uint32_t* status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = index[i];
    if ((int64_t)k >= n_targets) {
        old[i] = 0xFFFFFFFFu;
        __hip_atomic_fetch_or(status, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    uint32_t* x = target + k;
    const uint32_t v = e[i];
    uint32_t r = 0;
    switch (op) {
        case OMPRT_ATOMIC_ADD:
            r = __hip_atomic_fetch_add(x, v, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
            break;
        case OMPRT_ATOMIC_INC:
            r = __builtin_amdgcn_atomic_inc32(x, v, __ATOMIC_SEQ_CST, "agent");
            break;
        case OMPRT_ATOMIC_MAX:
            r = __hip_atomic_fetch_max(x, v, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
            break;
        case OMPRT_ATOMIC_EXCHANGE:
            r = __hip_atomic_exchange(x, v, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
            break;
        case OMPRT_ATOMIC_CAS: {
            uint32_t expected = v;   // on failure it receives the current value
            __hip_atomic_compare_exchange_strong(x, &expected, d[i], __ATOMIC_SEQ_CST,
                                                 __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
            r = expected;
            break;
        }
    }
    old[i] = r;
}

}  // namespace omprt

using namespace omprt;

extern "C" omprt_status omprt_atomic_apply(int32_t op, uint32_t* d_target, int64_t n_targets,
                                           const uint32_t* d_index, const uint32_t* d_e,
                                           const uint32_t* d_d, uint32_t* d_old, int64_t n,
                                           void* hip_stream) {
    if (op < OMPRT_ATOMIC_ADD || op > OMPRT_ATOMIC_CAS)
        return fail(OMPRT_ERR_INVALID, "atomic op %d", op);
    if (n < 0 || n > ((int64_t)1 << 40)) return fail(OMPRT_ERR_INVALID, "n = %lld", (long long)n);
    if (n == 0) return OMPRT_OK;
    if (n_targets < 1) return fail(OMPRT_ERR_INVALID, "n_targets < 1");
    if (!d_target || !d_index || !d_e || !d_old || (op == OMPRT_ATOMIC_CAS && !d_d))
        return fail(OMPRT_ERR_INVALID, "NULL pointer");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    Workspace* ws = nullptr;
    if (omprt_status st = workspace_get(stream, 1, &ws)) return st;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > INT32_MAX) return fail(OMPRT_ERR_INVALID, "n too large for one launch");
    hipLaunchKernelGGL(atomic_apply_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, (int)op,
                       d_target, n_targets, d_index, d_e, d_d, d_old, n, ws->status());
    OMPRT_HIP(hipGetLastError());
    return OMPRT_OK;
}
