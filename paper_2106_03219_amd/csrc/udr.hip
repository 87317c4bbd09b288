// udr.hip -- user-defined reductions (OpenMP's declare reduction): the
// reduction type, its initializer and its combiner are the user's code, so
// the kernel is compiled when the reduction is declared.  The runtime
// specialises its generic reduction with the application's code, the same
// move the paper makes by linking the device runtime into the application as
// bitcode (sec. 2.2), here done at run time with hiprtc.
//
// The generated kernel is the plain reduction's pipeline with the user's
// type: teams take the balanced block bal(n, T, k) of the input; lanes read
// interleaved 16-byte vectors, four in flight, and a lane folds its elements
// with the user's loop body into up to four private copies (one per element
// slot of a vector for types up to 32 bytes, each in increasing position;
// the head before 16-byte alignment and the tail one element a lane), which
// it then combines;
// private copies meet through
// the wave / team tree and the tagged last-team combine (a type of up to
// 64 bytes spans up to four cross-team slots); the last team combines the
// original value of the variable with the result.  The combiner is applied
// in an order the user cannot rely on, as OpenMP allows.
#include <hip/hiprtc.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "device.h"
#include "runtime.h"

#include "rtc_headers.inc"

namespace omprt {
namespace {

// What the run-time compiler sees for the system headers the device headers
// include: the fixed-width integer types come from hiprtc's own prelude.
const char* const kRtcStubHipRuntime = "#pragma once\n";
const char* const kRtcStubStdint =
    "#pragma once\n"
    "typedef __hip_internal::int8_t int8_t;\n"
    "typedef __hip_internal::uint8_t uint8_t;\n"
    "typedef __hip_internal::int16_t int16_t;\n"
    "typedef __hip_internal::uint16_t uint16_t;\n"
    "typedef __hip_internal::int32_t int32_t;\n"
    "typedef __hip_internal::uint32_t uint32_t;\n"
    "typedef __hip_internal::int64_t int64_t;\n"
    "typedef __hip_internal::uint64_t uint64_t;\n"
    "typedef unsigned long uintptr_t;\n"
    "#define INT32_MIN (-2147483647 - 1)\n"
    "#define INT32_MAX 2147483647\n"
    "#define INT64_MIN (-9223372036854775807LL - 1)\n"
    "#define INT64_MAX 9223372036854775807LL\n"
    "#define UINT32_MAX 4294967295u\n";

// The kernel around the user's code.  @DT@ is the input's dtype code,
// @BYTES@ the declared size of the type.
const char* const kUdrKernel = R"omprt_udr(
#include "device.h"
#include "stream.h"
namespace omprt_udr {
using namespace omprt;
#line 1 "omp_type"
@TYPE@
#line 1 "generated"
static_assert(sizeof(omp_type) == @BYTES@, "sizeof(omp_type) differs from the declared acc_bytes");
static_assert(sizeof(omp_type) % 4 == 0 && sizeof(omp_type) <= 64,
              "omp_type must be a multiple of 4 bytes, at most 64");
using Elem = DType<@DT@>;
struct Policy {
    using Acc = omp_type;
    static __device__ __forceinline__ Acc identity() {
        omp_type omp_priv;
#line 1 "initializer"
@INIT@
#line 1 "generated"
        return omp_priv;
    }
    static __device__ __forceinline__ Acc combine(Acc omp_out, const Acc omp_in_value) {
        const omp_type& omp_in = omp_in_value;
#line 1 "combiner"
@COMBINER@
#line 1 "generated"
        return omp_out;
    }
    static __device__ __forceinline__ void elem(Acc& omp_priv, const typename Elem::V omp_elem,
                                                const int64_t omp_i) {
#line 1 "body"
@BODY@
#line 1 "generated"
    }
};
}  // namespace omprt_udr

extern "C" __global__ __launch_bounds__(1024) void omprt_udr_kernel(
    const typename omprt_udr::Elem::S* __restrict__ in, int64_t n, omprt_udr::omp_type* x,
    omprt::CrossTeam ct) {
    using namespace omprt;
    using R = omprt_udr::Policy;
    using D = omprt_udr::Elem;
    using L = VecLoad<@DT@, 16>;
    using Vec = typename L::T;
    constexpr int PER = L::PER;
    constexpr int U = 4;
    __shared__ R::Acc lds[kMaxWaves];
    __shared__ int s_last;
    const int64_t T = gridDim.x;
    const int64_t P = blockDim.x;
    const int64_t tid = threadIdx.x;
    const uint32_t epoch = T > 1 ? read_epoch(ct.epoch) : 0u;
    const Range blk = bal_share(n, T, blockIdx.x);
    // A lane keeps one private copy per element slot of a vector (at most
    // four), each folding its elements in increasing position, and combines
    // them at the end: independent update chains instead of one (an exact
    // three-field int32 reduction: 5.2 -> 6.5 TB/s).  Types over 32 bytes keep
    // one copy: several copies of a 64-byte type with an indexed member went
    // to scratch memory (6.7 -> 0.95 TB/s).
    constexpr int NA = sizeof(R::Acc) > 32 ? 1 : PER < 4 ? PER : 4;
    R::Acc acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = R::identity();
    if (blk.lo < blk.hi) {
        // the head up to 16-byte alignment, the vectors (lanes interleaved), the tail
        const int64_t lo = blk.lo, hi = blk.hi;
        const uintptr_t mis = reinterpret_cast<uintptr_t>(in + lo) & 15;
        int64_t head = (int64_t)(((16 - mis) & 15) / sizeof(typename D::S));
        if (head > hi - lo) head = hi - lo;
        if (tid < head) R::elem(acc[0], D::from(in[lo + tid]), lo + tid);
        const int64_t p0 = lo + head;
        const int64_t nv = (hi - p0) / PER;
        const Vec* __restrict__ vp = reinterpret_cast<const Vec*>(in + p0);
        int64_t v = tid;
        for (; v + (U - 1) * P < nv; v += U * P) {
            Vec r[U];
#pragma unroll
            for (int u = 0; u < U; ++u) r[u] = L::load(vp + v + u * P);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i0 = p0 + (v + u * P) * PER;
#pragma unroll
                for (int e = 0; e < PER; ++e) R::elem(acc[e % NA], L::get(r[u], e), i0 + e);
            }
        }
        for (; v < nv; v += P) {
            const Vec r = L::load(vp + v);
            const int64_t i0 = p0 + v * PER;
#pragma unroll
            for (int e = 0; e < PER; ++e) R::elem(acc[e % NA], L::get(r, e), i0 + e);
        }
        const int64_t t0 = p0 + nv * PER;
        if (tid < hi - t0) R::elem(acc[0], D::from(in[t0 + tid]), t0 + tid);
    }
    R::Acc a = acc[0];
#pragma unroll
    for (int q = 1; q < NA; ++q) a = R::combine(a, acc[q]);
    a = team_reduce<R>(a, lds);
    R::Acc c = a;
    if (T > 1) {
        const uint32_t tag = launch_tag(epoch);
        if (!publish_and_elect(a, ct.slots + (size_t)blockIdx.x * slot_words<R::Acc>(), ct.counter,
                               (uint32_t)(T - 1), tag, &s_last))
            return;
        c = combine_slots<R>(ct.slots, T, tag, ct.status, lds);
    }
    if (threadIdx.x == 0) {
        x[0] = R::combine(x[0], c);
        if (T > 1) advance_epoch(ct.epoch, epoch);
    }
}
)omprt_udr";

constexpr const char* kUdrArch = "gfx950";
constexpr size_t kMaxLog = 1500;   // characters of compiler output kept in the error

struct UdrProgram {
    std::string key;    // dtype, size and source: a repeated declaration reuses the program
    int dtype = 0;
    int acc_bytes = 0;
    std::vector<char> code;   // gfx950 code object
};

std::mutex g_udr_mu;
std::vector<UdrProgram> g_udr;                                        // handle = index
std::map<std::pair<int, int>, std::pair<hipModule_t, hipFunction_t>> g_udr_fn;   // (handle, dev)

void replace_all(std::string& s, const std::string& what, const std::string& with) {
    for (size_t p = s.find(what); p != std::string::npos; p = s.find(what, p + with.size()))
        s.replace(p, what.size(), with);
}

omprt_status compile_udr(const std::string& src, std::vector<char>* code) {
    const char* names[kRtcHeaderCount + 2];
    const char* texts[kRtcHeaderCount + 2];
    names[0] = "hip/hip_runtime.h";
    texts[0] = kRtcStubHipRuntime;
    names[1] = "stdint.h";
    texts[1] = kRtcStubStdint;
    for (int h = 0; h < kRtcHeaderCount; ++h) {
        names[h + 2] = kRtcHeaderNames[h];
        texts[h + 2] = kRtcHeaderTexts[h];
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "omprt_udr.hip", kRtcHeaderCount + 2, texts,
                            names) != HIPRTC_SUCCESS)
        return fail(OMPRT_ERR_DEVICE, "declare reduction: hiprtcCreateProgram failed");
    const std::string arch = std::string("--offload-arch=") + kUdrArch;
    // no packed-fp32 VALU instructions, as for the rest of the library
    const char* opts[] = {arch.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, 7, opts);
    size_t log_size = 0;
    std::string log;
    if (hiprtcGetProgramLogSize(prog, &log_size) == HIPRTC_SUCCESS && log_size > 1) {
        log.resize(log_size);
        if (hiprtcGetProgramLog(prog, &log[0]) != HIPRTC_SUCCESS) log.clear();
    }
    omprt_status st = OMPRT_OK;
    if (r != HIPRTC_SUCCESS) {
        if (log.size() > kMaxLog) log = log.substr(0, kMaxLog) + " ...";
        st = fail(OMPRT_ERR_INVALID, "declare reduction: the user's code does not compile:\n%s",
                  log.c_str());
    } else {
        size_t n = 0;
        if (hiprtcGetCodeSize(prog, &n) != HIPRTC_SUCCESS || n == 0) {
            st = fail(OMPRT_ERR_DEVICE, "declare reduction: no code object");
        } else {
            code->resize(n);
            if (hiprtcGetCode(prog, code->data()) != HIPRTC_SUCCESS)
                st = fail(OMPRT_ERR_DEVICE, "declare reduction: hiprtcGetCode failed");
        }
    }
    hiprtcDestroyProgram(&prog);
    return st;
}

// The kernel of `handle` on the current device, loading its module on first use.
omprt_status udr_function(int handle, hipFunction_t* f, int* acc_bytes, int* dtype) {
    int dev = 0;
    OMPRT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_udr_mu);
    if (handle < 0 || handle >= (int)g_udr.size())
        return fail(OMPRT_ERR_INVALID, "unknown user-defined reduction %d", handle);
    const UdrProgram& p = g_udr[handle];
    *acc_bytes = p.acc_bytes;
    *dtype = p.dtype;
    auto it = g_udr_fn.find({handle, dev});
    if (it != g_udr_fn.end()) {
        *f = it->second.second;
        return OMPRT_OK;
    }
    hipDeviceProp_t prop;
    OMPRT_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::string(prop.gcnArchName).rfind(kUdrArch, 0) != 0)
        return fail(OMPRT_ERR_UNSUPPORTED, "device %d is %s; user-defined reductions are built for %s",
                    dev, prop.gcnArchName, kUdrArch);
    hipModule_t mod;
    OMPRT_HIP(hipModuleLoadData(&mod, p.code.data()));
    hipFunction_t fn;
    const hipError_t e = hipModuleGetFunction(&fn, mod, "omprt_udr_kernel");
    if (e != hipSuccess) {
        (void)hipModuleUnload(mod);
        return fail(OMPRT_ERR_DEVICE, "hipModuleGetFunction: %s", hipGetErrorString(e));
    }
    g_udr_fn[{handle, dev}] = {mod, fn};
    *f = fn;
    return OMPRT_OK;
}

}  // namespace

void udr_finalize() {
    std::lock_guard<std::mutex> lk(g_udr_mu);
    int dev = 0;
    const bool have_dev = hipGetDevice(&dev) == hipSuccess;
    for (auto& kv : g_udr_fn) {
        (void)hipSetDevice(kv.first.second);
        (void)hipModuleUnload(kv.second.first);
    }
    g_udr_fn.clear();
    if (have_dev) (void)hipSetDevice(dev);
}

}  // namespace omprt

using namespace omprt;

extern "C" omprt_status omprt_udr_declare(const omprt_udr_source* src, int32_t dtype,
                                          int32_t* h_handle) {
    if (!src || !h_handle) return fail(OMPRT_ERR_INVALID, "source or handle is NULL");
    if (dtype < 0 || dtype >= DT_COUNT_ABI) return fail(OMPRT_ERR_UNSUPPORTED, "dtype %d", dtype);
    if (!src->type_def || !src->initializer || !src->combiner || !src->body)
        return fail(OMPRT_ERR_INVALID, "type_def, initializer, combiner and body are required");
    if (src->acc_bytes < 4 || src->acc_bytes > 64 || src->acc_bytes % 4)
        return fail(OMPRT_ERR_INVALID, "acc_bytes %d: 4..64, a multiple of 4", src->acc_bytes);
    std::string code = kUdrKernel;
    replace_all(code, "@DT@", std::to_string(dtype));
    replace_all(code, "@BYTES@", std::to_string(src->acc_bytes));
    // the user's text last, so that markers inside it are left alone
    const std::string mark(1, '\x01');
    replace_all(code, "@TYPE@", mark + "TYPE");
    replace_all(code, "@INIT@", mark + "INIT");
    replace_all(code, "@COMBINER@", mark + "COMB");
    replace_all(code, "@BODY@", mark + "BODY");
    std::string out;
    out.reserve(code.size() + 4096);
    for (size_t i = 0; i < code.size(); ++i) {
        if (code[i] == '\x01') {
            const std::string tag = code.substr(i + 1, 4);
            out += tag == "TYPE" ? src->type_def
                 : tag == "INIT" ? src->initializer
                 : tag == "COMB" ? src->combiner
                                 : src->body;
            i += 4;
        } else {
            out += code[i];
        }
    }
    const std::string key = std::to_string(dtype) + '\0' + std::to_string(src->acc_bytes) + '\0' +
                            src->type_def + '\0' + src->initializer + '\0' + src->combiner + '\0' +
                            src->body;
    {
        std::lock_guard<std::mutex> lk(g_udr_mu);
        for (size_t h = 0; h < g_udr.size(); ++h)
            if (g_udr[h].key == key) {
                *h_handle = (int32_t)h;
                return OMPRT_OK;
            }
    }
    UdrProgram p;
    if (omprt_status st = compile_udr(out, &p.code)) return st;
    p.key = key;
    p.dtype = dtype;
    p.acc_bytes = src->acc_bytes;
    std::lock_guard<std::mutex> lk(g_udr_mu);
    g_udr.push_back(std::move(p));
    *h_handle = (int32_t)(g_udr.size() - 1);
    return OMPRT_OK;
}

extern "C" omprt_status omprt_reduce_udr(int32_t handle, const void* d_in, int64_t n, void* d_x,
                                         const omprt_config* cfg, void* hip_stream) {
    if (n < 0 || n > ((int64_t)1 << 50))
        return fail(OMPRT_ERR_INVALID, "n = %lld outside 0..2^50", (long long)n);
    if (!d_x) return fail(OMPRT_ERR_INVALID, "x is NULL");
    if (n > 0 && !d_in) return fail(OMPRT_ERR_INVALID, "input is NULL with n > 0");
    int acc_bytes = 0, dtype = 0;
    {
        std::lock_guard<std::mutex> lk(g_udr_mu);
        if (handle < 0 || handle >= (int)g_udr.size())
            return fail(OMPRT_ERR_INVALID, "unknown user-defined reduction %d", handle);
        acc_bytes = g_udr[handle].acc_bytes;
        dtype = g_udr[handle].dtype;
    }
    if (reinterpret_cast<uintptr_t>(d_in) % dtype_bytes(dtype))
        return fail(OMPRT_ERR_INVALID, "input is not aligned to its element size");
    if (reinterpret_cast<uintptr_t>(d_x) % 4) return fail(OMPRT_ERR_INVALID, "x is not 4-byte aligned");
    if (cfg && (cfg->vec_bytes || cfg->unroll))
        return fail(OMPRT_ERR_INVALID, "user-defined reductions take num_teams and threads_per_team only");
    omprt_config c2 = cfg ? *cfg : omprt_config{};
    c2.flags |= OMPRT_CFG_NO_MODEL;
    LaunchCfg lc;
    if (omprt_status st = resolve_config(n, dtype, OP_SUM, 0, -1, &c2, &lc, nullptr)) return st;
    if (n == 0) return OMPRT_OK;
    const int slots = (acc_bytes / 4 + kSlotWords - 1) / kSlotWords;
    if ((int64_t)lc.teams * slots > 65535 * 4)
        return fail(OMPRT_ERR_INVALID, "num_teams %d too large for %d-byte partials", lc.teams,
                    acc_bytes);
    hipFunction_t f;
    if (omprt_status st = udr_function(handle, &f, &acc_bytes, &dtype)) return st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    Workspace* ws = nullptr;
    if (omprt_status st = workspace_get(stream, lc.teams * slots, &ws)) return st;
    const CrossTeamArgs ca = ws->cross();
    CrossTeam ct{static_cast<uint64_t*>(ca.slots), ca.counter, ca.epoch, ca.status};
    void* args[] = {&d_in, &n, &d_x, &ct};
    OMPRT_HIP(hipModuleLaunchKernel(f, lc.teams, 1, 1, lc.threads, 1, 1, 0, stream, args, nullptr));
    return OMPRT_OK;
}
