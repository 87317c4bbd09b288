// mlp.hip -- the learned configuration picker's network on the GPU:
// forward (logits), mean softmax cross-entropy with its full backward pass,
// and the Adam update, in fp32.  Shapes are tiny (F = 16, H = 64, K <= 64,
// batches of a few hundred to tens of thousands of rows), so every kernel is
// a plain one-thread-per-output VALU kernel; sums over batch rows use TwoSum
// compensation so the gradients track an FP64 reference closely.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "device.h"
#include "runtime.h"

namespace omprt {

// Y[r][j] = act(b[j] + sum_i W[j][i] X[r][i])
__global__ void mlp_linear_kernel(const float* __restrict__ X, const float* __restrict__ W,
                                  const float* __restrict__ b, float* __restrict__ Y, int B,
                                  int in, int out, int relu) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * out) return;
    const int r = (int)(idx / out), j = (int)(idx % out);
    float s = b[j];
    const float* w = W + (int64_t)j * in;
    const float* x = X + (int64_t)r * in;
    for (int i = 0; i < in; ++i) s = __builtin_fmaf(w[i], x[i], s);
    Y[idx] = relu ? fmaxf(s, 0.0f) : s;
}

// Per row: loss_r = logsumexp(z) - z[y];  dZ[r][j] = (softmax(z)_j - [j == y]) / B.
// One wave per row, lanes over the classes (max and sum by wave reductions).
struct MaxPolicy {
    using Acc = float;
    static __device__ __forceinline__ float combine(float a, float b) { return fmaxf(a, b); }
};
struct AddPolicy {
    using Acc = float;
    static __device__ __forceinline__ float combine(float a, float b) { return a + b; }
};
__global__ __launch_bounds__(256) void mlp_softmax_ce_kernel(const float* __restrict__ Z,
                                                             const int32_t* __restrict__ y,
                                                             float* __restrict__ dZ,
                                                             float* __restrict__ row_loss, int B,
                                                             int K) {
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (r >= B) return;   // whole waves
    const float* z = Z + r * K;
    float mx = -INFINITY;
    for (int j = lane; j < K; j += kWave) mx = fmaxf(mx, z[j]);
    mx = wave_reduce<MaxPolicy>(mx);
    float den = 0.0f;
    for (int j = lane; j < K; j += kWave) den += expf(z[j] - mx);
    den = wave_reduce<AddPolicy>(den);
    const int lab = y[r];
    if (lane == 0) row_loss[r] = logf(den) - (z[lab] - mx);
    const float inv = 1.0f / (float)B;
    for (int j = lane; j < K; j += kWave) {
        const float p = expf(z[j] - mx) / den;
        dZ[r * K + j] = (p - (j == lab ? 1.0f : 0.0f)) * inv;
    }
}

// GW[j][i] = sum_r D[r][j] A[r][i];  gb[j] = sum_r D[r][j]   (compensated over r;
// the product is rounded on its own so it is not fused into the TwoSum).  One
// wave per output: lane l takes rows l, l + 64, ..., and the lanes' pairs
// combine through the wave's float-float tree.
struct PairPolicy {
    using Acc = ff_t;
    static __device__ __forceinline__ ff_t combine(ff_t a, ff_t b) { return pair_add(a, b); }
};
__global__ __launch_bounds__(256) void mlp_weight_grad_kernel(const float* __restrict__ D,
                                                              const float* __restrict__ A,
                                                              float* __restrict__ GW,
                                                              float* __restrict__ gb, int B,
                                                              int out, int in) {
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (w >= (int64_t)out * (in + 1)) return;   // whole waves
    const int j = (int)(w / (in + 1)), i = (int)(w % (in + 1));
    ff_t acc{0.0f, 0.0f};
    if (i == in) {
        for (int r = lane; r < B; r += kWave) comp_add(acc, D[(int64_t)r * out + j]);
    } else {
        for (int r = lane; r < B; r += kWave)
            comp_add(acc, __fmul_rn(D[(int64_t)r * out + j], A[(int64_t)r * in + i]));
    }
    acc = wave_reduce<PairPolicy>(acc);
    if (lane == 0) {
        if (i == in)
            gb[j] = acc.hi + acc.lo;
        else
            GW[(int64_t)j * in + i] = acc.hi + acc.lo;
    }
}

// Dprev[r][i] = (sum_j D[r][j] W[j][i]) * [Aprev[r][i] > 0]
__global__ void mlp_backprop_kernel(const float* __restrict__ D, const float* __restrict__ W,
                                    const float* __restrict__ Aprev, float* __restrict__ Dprev,
                                    int B, int out, int in) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * in) return;
    const int r = (int)(idx / in), i = (int)(idx % in);
    float s = 0.0f;
    const float* d = D + (int64_t)r * out;
    for (int j = 0; j < out; ++j) s = __builtin_fmaf(d[j], W[(int64_t)j * in + i], s);
    Dprev[idx] = Aprev[idx] > 0.0f ? s : 0.0f;
}

// out[0] = mean of v[0..B) (one workgroup of 256; fixed order; compensated)
struct MeanPolicy : CompSum<float, 1> {};
__global__ __launch_bounds__(256) void mlp_mean_kernel(const float* __restrict__ v, int B,
                                                       float* __restrict__ out) {
    __shared__ ff_t slots[kMaxWaves];
    ff_t acc{0.0f, 0.0f};
    for (int i = threadIdx.x; i < B; i += blockDim.x) comp_add(acc, v[i]);
    acc = team_reduce<MeanPolicy>(acc, slots);
    if (threadIdx.x == 0) out[0] = (acc.hi + acc.lo) / (float)B;
}

__global__ void mlp_adam_kernel(float* __restrict__ w, float* __restrict__ m,
                                float* __restrict__ v, const float* __restrict__ g, int64_t n,
                                float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Adam with the step count in device memory: t = *step + 1 (the bias
// corrections are computed per thread, in double as the host path does, so
// the update is bit for bit the one omprt_mlp_adam makes at step t).
__global__ void mlp_adam_counted_kernel(float* __restrict__ w, float* __restrict__ m,
                                        float* __restrict__ v, const float* __restrict__ g,
                                        int64_t n, const int32_t* __restrict__ step, float lr,
                                        float b1, float b2, float eps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t = (double)step[0] + 1.0;
    const float c1 = (float)(1.0 - pow((double)b1, t));
    const float c2 = (float)(1.0 - pow((double)b2, t));
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void mlp_step_advance_kernel(int32_t* step) { step[0] += 1; }

// ---------------------------------------------------------------- scratch

struct MlpScratch {
    float* base = nullptr;
    int64_t floats = 0;
};
static std::mutex g_mmu;
static std::map<std::pair<int, hipStream_t>, MlpScratch> g_mscr;

static omprt_status mlp_scratch(hipStream_t s, int64_t floats, float** out) {
    int dev = 0;
    OMPRT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mmu);
    MlpScratch& m = g_mscr[{dev, s}];
    if (m.floats < floats) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        OMPRT_HIP(hipStreamIsCapturing(s, &cs));
        if (cs != hipStreamCaptureStatusNone)
            return fail(OMPRT_ERR_INVALID, "MLP scratch must grow outside stream capture");
        float* q = nullptr;
        if (hipMalloc(&q, sizeof(float) * (size_t)floats) != hipSuccess)
            return fail(OMPRT_ERR_NOMEM, "MLP scratch allocation failed");
        retire_device_memory(dev, m.base);   // a captured graph may still name it
        m.base = q;
        m.floats = floats;
    }
    *out = m.base;
    return OMPRT_OK;
}

void mlp_finalize() {
    std::lock_guard<std::mutex> lk(g_mmu);
    for (auto& kv : g_mscr) {
        if (!kv.second.base) continue;
        (void)hipSetDevice(kv.first.first);
        (void)hipFree(kv.second.base);
    }
    g_mscr.clear();
}

static omprt_status check_dims(const omprt_mlp_dims* d) {
    if (!d) return fail(OMPRT_ERR_INVALID, "dims is NULL");
    if (d->F < 1 || d->H1 < 1 || d->H2 < 1 || d->K < 2 || d->F > 4096 || d->H1 > 4096 ||
        d->H2 > 4096 || d->K > 4096)
        return fail(OMPRT_ERR_INVALID, "MLP dims out of range");
    return OMPRT_OK;
}

static inline unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace omprt

using namespace omprt;

extern "C" int64_t omprt_mlp_param_count(const omprt_mlp_dims* d) {
    if (!d) return -1;
    return (int64_t)d->H1 * d->F + d->H1 + (int64_t)d->H2 * d->H1 + d->H2 +
           (int64_t)d->K * d->H2 + d->K;
}

struct ParamView {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};
static ParamView view(const omprt_mlp_dims* d, const float* p) {
    ParamView v;
    v.W1 = p;
    v.b1 = v.W1 + (int64_t)d->H1 * d->F;
    v.W2 = v.b1 + d->H1;
    v.b2 = v.W2 + (int64_t)d->H2 * d->H1;
    v.W3 = v.b2 + d->H2;
    v.b3 = v.W3 + (int64_t)d->K * d->H2;
    return v;
}

extern "C" omprt_status omprt_mlp_forward(const omprt_mlp_dims* d, const float* d_params,
                                          const float* d_X, int32_t B, float* d_Z,
                                          void* hip_stream) {
    if (omprt_status st = check_dims(d)) return st;
    if (B < 0 || B > 65536) return fail(OMPRT_ERR_INVALID, "B outside 0..65536");
    if (B == 0) return OMPRT_OK;
    if (!d_params || !d_X || !d_Z) return fail(OMPRT_ERR_INVALID, "NULL pointer");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    float* scr = nullptr;
    if (omprt_status st = mlp_scratch(s, (int64_t)B * (d->H1 + d->H2), &scr)) return st;
    float* a1 = scr;
    float* a2 = a1 + (int64_t)B * d->H1;
    const ParamView p = view(d, d_params);
    hipLaunchKernelGGL(mlp_linear_kernel, dim3(blocks((int64_t)B * d->H1, 256)), dim3(256), 0, s,
                       d_X, p.W1, p.b1, a1, B, d->F, d->H1, 1);
    hipLaunchKernelGGL(mlp_linear_kernel, dim3(blocks((int64_t)B * d->H2, 256)), dim3(256), 0, s,
                       a1, p.W2, p.b2, a2, B, d->H1, d->H2, 1);
    hipLaunchKernelGGL(mlp_linear_kernel, dim3(blocks((int64_t)B * d->K, 256)), dim3(256), 0, s,
                       a2, p.W3, p.b3, d_Z, B, d->H2, d->K, 0);
    OMPRT_HIP(hipGetLastError());
    return OMPRT_OK;
}

extern "C" omprt_status omprt_mlp_loss_grad(const omprt_mlp_dims* d, const float* d_params,
                                            const float* d_X, const int32_t* d_y, int32_t B,
                                            float* d_loss, float* d_grads, void* hip_stream) {
    if (omprt_status st = check_dims(d)) return st;
    if (B < 1 || B > 65536) return fail(OMPRT_ERR_INVALID, "B outside 1..65536");
    if (!d_params || !d_X || !d_y || !d_loss || !d_grads)
        return fail(OMPRT_ERR_INVALID, "NULL pointer");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int64_t H1 = d->H1, H2 = d->H2, K = d->K, F = d->F;
    float* scr = nullptr;
    const int64_t need = (int64_t)B * (2 * H1 + 2 * H2 + 2 * K + 1);
    if (omprt_status st = mlp_scratch(s, need, &scr)) return st;
    float* a1 = scr;
    float* a2 = a1 + B * H1;
    float* z = a2 + B * H2;
    float* dz = z + B * K;
    float* d2 = dz + B * K;
    float* d1 = d2 + B * H2;
    float* rl = d1 + B * H1;
    const ParamView p = view(d, d_params);
    float* gW1 = d_grads;
    float* gb1 = gW1 + H1 * F;
    float* gW2 = gb1 + H1;
    float* gb2 = gW2 + H2 * H1;
    float* gW3 = gb2 + H2;
    float* gb3 = gW3 + K * H2;
    hipLaunchKernelGGL(mlp_linear_kernel, dim3(blocks(B * H1, 256)), dim3(256), 0, s, d_X, p.W1,
                       p.b1, a1, B, (int)F, (int)H1, 1);
    hipLaunchKernelGGL(mlp_linear_kernel, dim3(blocks(B * H2, 256)), dim3(256), 0, s, a1, p.W2,
                       p.b2, a2, B, (int)H1, (int)H2, 1);
    hipLaunchKernelGGL(mlp_linear_kernel, dim3(blocks(B * K, 256)), dim3(256), 0, s, a2, p.W3,
                       p.b3, z, B, (int)H2, (int)K, 0);
    hipLaunchKernelGGL(mlp_softmax_ce_kernel, dim3(blocks((int64_t)B * kWave, 256)), dim3(256), 0,
                       s, z, d_y, dz, rl, B, (int)K);
    hipLaunchKernelGGL(mlp_mean_kernel, dim3(1), dim3(256), 0, s, rl, B, d_loss);
    hipLaunchKernelGGL(mlp_weight_grad_kernel, dim3(blocks(K * (H2 + 1) * kWave, 256)), dim3(256),
                       0, s, dz, a2, gW3, gb3, B, (int)K, (int)H2);
    hipLaunchKernelGGL(mlp_backprop_kernel, dim3(blocks(B * H2, 256)), dim3(256), 0, s, dz, p.W3,
                       a2, d2, B, (int)K, (int)H2);
    hipLaunchKernelGGL(mlp_weight_grad_kernel, dim3(blocks(H2 * (H1 + 1) * kWave, 256)),
                       dim3(256), 0, s, d2, a1, gW2, gb2, B, (int)H2, (int)H1);
    hipLaunchKernelGGL(mlp_backprop_kernel, dim3(blocks(B * H1, 256)), dim3(256), 0, s, d2, p.W2,
                       a1, d1, B, (int)H2, (int)H1);
    hipLaunchKernelGGL(mlp_weight_grad_kernel, dim3(blocks(H1 * (F + 1) * kWave, 256)), dim3(256),
                       0, s, d1, d_X, gW1, gb1, B, (int)H1, (int)F);
    OMPRT_HIP(hipGetLastError());
    return OMPRT_OK;
}

extern "C" omprt_status omprt_mlp_adam(float* d_params, float* d_m, float* d_v,
                                       const float* d_grads, int64_t n, int32_t step, float lr,
                                       float beta1, float beta2, float eps, void* hip_stream) {
    if (n < 0 || step < 1) return fail(OMPRT_ERR_INVALID, "n < 0 or step < 1");
    if (n == 0) return OMPRT_OK;
    if (!d_params || !d_m || !d_v || !d_grads) return fail(OMPRT_ERR_INVALID, "NULL pointer");
    const float c1 = (float)(1.0 - pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - pow((double)beta2, (double)step));
    hipLaunchKernelGGL(mlp_adam_kernel, dim3(blocks(n, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), d_params, d_m, d_v, d_grads, n, lr,
                       beta1, beta2, eps, c1, c2);
    OMPRT_HIP(hipGetLastError());
    return OMPRT_OK;
}

extern "C" omprt_status omprt_mlp_adam_counted(float* d_params, float* d_m, float* d_v,
                                               const float* d_grads, int64_t n, int32_t* d_step,
                                               float lr, float beta1, float beta2, float eps,
                                               void* hip_stream) {
    if (n < 0) return fail(OMPRT_ERR_INVALID, "n < 0");
    if (!d_step) return fail(OMPRT_ERR_INVALID, "step counter is NULL");
    if (n == 0) return OMPRT_OK;
    if (!d_params || !d_m || !d_v || !d_grads) return fail(OMPRT_ERR_INVALID, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(d_step) & 3)
        return fail(OMPRT_ERR_INVALID, "step counter not 4-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(mlp_adam_counted_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, d_params,
                       d_m, d_v, d_grads, n, d_step, lr, beta1, beta2, eps);
    hipLaunchKernelGGL(mlp_step_advance_kernel, dim3(1), dim3(1), 0, s, d_step);
    OMPRT_HIP(hipGetLastError());
    return OMPRT_OK;
}
