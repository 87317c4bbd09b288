// model.hip -- host side of the learned configuration picker: call
// features, the weight-file loader, and per-call CPU inference of the small
// MLP (about 10k multiply-adds) with a confidence threshold.  A call the
// model is not confident about falls back to the tuned cache / heuristic.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <unordered_map>
#include <string>
#include <vector>

#include "runtime.h"

namespace omprt {

struct ClassCfg {
    int teams_per_cu, threads, vec, unroll;
};

struct Model {
    int F = 0, H1 = 0, H2 = 0, K = 0;
    float tau = 0.0f;
    std::vector<float> mean, scale, params;
    std::vector<ClassCfg> classes;
};

static std::mutex g_model_mu;
static Model* g_model = nullptr;

static float log2f_pos(double v) { return v > 0 ? (float)log2(v) : 0.0f; }

// f0 log2 n; f1..f5 dtype one-hot (i32, i64, f32, f64, bf16); f6..f8 op
// one-hot; f9 log2 chunk (0 if none/default); f10 chunk given as 0; f11
// bytes per iteration; f12 flops per iteration; f13 log2 total bytes; f14
// compensated accumulation; f15 user chunk given.
void model_features(int64_t n, int dtype, int op, int body, int64_t chunk, float* f) {
    for (int i = 0; i < 16; ++i) f[i] = 0.0f;
    const int eb = body ? 12 : dtype_bytes(dtype);
    f[0] = log2f_pos((double)n);
    if (dtype >= 0 && dtype < 5) f[1 + dtype] = 1.0f;
    if (op >= 0 && op < 3) f[6 + op] = 1.0f;
    f[9] = chunk > 0 ? log2f_pos((double)chunk) : 0.0f;
    f[10] = chunk == 0 ? 1.0f : 0.0f;
    f[11] = (float)eb;
    f[12] = body ? 2.0f : (op == OMPRT_SUM && (dtype == OMPRT_F32 || dtype == OMPRT_BF16) ? 4.0f : 1.0f);
    f[13] = log2f_pos((double)n * eb);
    f[14] = (op == OMPRT_SUM && dtype != OMPRT_I32 && dtype != OMPRT_I64) ? 1.0f : 0.0f;
    f[15] = chunk >= 0 ? 1.0f : 0.0f;
}

// teams for a class: capped by teams_per_cu * CUs and by the work (one team
// per threads * vec bytes, at least 1)
static int class_teams(const ClassCfg& c, int64_t n, int eb) {
    const int64_t per = (int64_t)c.threads * c.vec;
    const int64_t work = (n * eb + per - 1) / per;
    int64_t t = (int64_t)c.teams_per_cu * device_cus();
    if (work < t) t = work;
    if (t < 1) t = 1;
    if (t > 65535) t = 65535;
    return (int)t;
}

// Decisions of the loaded model, keyed by the exact call properties, so a
// repeated call skips the host forward pass (cleared when a model is loaded).
struct PickKey {
    int64_t n, chunk;
    int dtype, op, body;
    bool operator==(const PickKey& o) const {
        return n == o.n && chunk == o.chunk && dtype == o.dtype && op == o.op && body == o.body;
    }
};
struct PickKeyHash {
    size_t operator()(const PickKey& k) const {
        uint64_t h = (uint64_t)k.n * 0x9E3779B97F4A7C15ull;
        h ^= (uint64_t)k.chunk + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
        h ^= (uint64_t)(k.dtype * 16 + k.op * 4 + k.body) + (h << 6) + (h >> 2);
        return (size_t)h;
    }
};
struct PickVal {
    bool have;
    LaunchCfg cfg;
};
static std::unordered_map<PickKey, PickVal, PickKeyHash> g_pick_cache;
constexpr size_t kPickCacheMax = 1 << 16;

static bool model_forward_pick(const Model* m, const float* f16, int body, int64_t n,
                               LaunchCfg* out);

bool model_pick(int64_t n, int dtype, int op, int body, int64_t chunk, LaunchCfg* out) {
    std::lock_guard<std::mutex> lk(g_model_mu);
    const Model* m = g_model;
    if (!m) return false;
    const PickKey key{n, chunk, dtype, op, body};
    auto it = g_pick_cache.find(key);
    if (it != g_pick_cache.end()) {
        if (it->second.have) *out = it->second.cfg;
        return it->second.have;
    }
    float f[16];
    model_features(n, dtype, op, body, chunk, f);
    PickVal v{false, LaunchCfg{}};
    v.have = model_forward_pick(m, f, body, n, &v.cfg);
    if (g_pick_cache.size() >= kPickCacheMax) g_pick_cache.clear();
    g_pick_cache.emplace(key, v);
    if (v.have) *out = v.cfg;
    return v.have;
}

static bool model_forward_pick(const Model* m, const float* f16, int body, int64_t n,
                               LaunchCfg* out) {
    float x[16], h1[4096], h2[4096], z[4096];
    for (int i = 0; i < m->F; ++i) x[i] = (f16[i] - m->mean[i]) * m->scale[i];
    const float* W1 = m->params.data();
    const float* b1 = W1 + m->H1 * m->F;
    const float* W2 = b1 + m->H1;
    const float* b2 = W2 + m->H2 * m->H1;
    const float* W3 = b2 + m->H2;
    const float* b3 = W3 + m->K * m->H2;
    for (int j = 0; j < m->H1; ++j) {
        float s = b1[j];
        for (int i = 0; i < m->F; ++i) s += W1[j * m->F + i] * x[i];
        h1[j] = s > 0 ? s : 0;
    }
    for (int j = 0; j < m->H2; ++j) {
        float s = b2[j];
        for (int i = 0; i < m->H1; ++i) s += W2[j * m->H1 + i] * h1[i];
        h2[j] = s > 0 ? s : 0;
    }
    int best = 0;
    for (int j = 0; j < m->K; ++j) {
        float s = b3[j];
        for (int i = 0; i < m->H2; ++i) s += W3[j * m->H2 + i] * h2[i];
        z[j] = s;
        if (z[j] > z[best]) best = j;
    }
    double den = 0.0;
    for (int j = 0; j < m->K; ++j) den += exp((double)(z[j] - z[best]));
    const double pmax = 1.0 / den;
    if (pmax < m->tau) return false;
    const ClassCfg& c = m->classes[best];
    const int eb = body ? 12 : (int)f16[11];
    out->teams = class_teams(c, n, eb);
    out->threads = c.threads;
    out->vec = c.vec;
    out->unroll = c.unroll;
    return true;
}

static omprt_status parse(FILE* fp, Model* m) {
    char magic[32] = {0};
    int ver = 0;
    if (fscanf(fp, "%31s %d", magic, &ver) != 2 || strcmp(magic, "omprt-mlp") != 0 || ver != 1)
        return fail(OMPRT_ERR_INVALID, "model file: bad header");
    char key[32];
    if (fscanf(fp, "%31s %d %d %d %d", key, &m->F, &m->H1, &m->H2, &m->K) != 5 ||
        strcmp(key, "dims") != 0 || m->F != 16 || m->H1 < 1 || m->H1 > 4096 || m->H2 < 1 ||
        m->H2 > 4096 || m->K < 2 || m->K > 4096)
        return fail(OMPRT_ERR_INVALID, "model file: bad dims");
    if (fscanf(fp, "%31s %f", key, &m->tau) != 2 || strcmp(key, "tau") != 0)
        return fail(OMPRT_ERR_INVALID, "model file: bad tau");
    m->mean.resize(16);
    m->scale.resize(16);
    if (fscanf(fp, "%31s", key) != 1 || strcmp(key, "mean") != 0)
        return fail(OMPRT_ERR_INVALID, "model file: missing mean");
    for (float& v : m->mean)
        if (fscanf(fp, "%f", &v) != 1) return fail(OMPRT_ERR_INVALID, "model file: bad mean");
    if (fscanf(fp, "%31s", key) != 1 || strcmp(key, "scale") != 0)
        return fail(OMPRT_ERR_INVALID, "model file: missing scale");
    for (float& v : m->scale)
        if (fscanf(fp, "%f", &v) != 1) return fail(OMPRT_ERR_INVALID, "model file: bad scale");
    if (fscanf(fp, "%31s", key) != 1 || strcmp(key, "classes") != 0)
        return fail(OMPRT_ERR_INVALID, "model file: missing classes");
    m->classes.resize((size_t)m->K);
    for (ClassCfg& c : m->classes) {
        if (fscanf(fp, "%d %d %d %d", &c.teams_per_cu, &c.threads, &c.vec, &c.unroll) != 4 ||
            c.teams_per_cu < 1 || c.threads < 64 || c.threads > 1024 || c.threads % 64 ||
            (c.vec != 8 && c.vec != 16) ||
            !(c.unroll == 1 || c.unroll == 2 || c.unroll == 4 || c.unroll == 8))
            return fail(OMPRT_ERR_INVALID, "model file: bad class row");
    }
    long long np = 0;
    if (fscanf(fp, "%31s %lld", key, &np) != 2 || strcmp(key, "params") != 0)
        return fail(OMPRT_ERR_INVALID, "model file: missing params");
    const long long want = (long long)m->H1 * m->F + m->H1 + (long long)m->H2 * m->H1 + m->H2 +
                           (long long)m->K * m->H2 + m->K;
    if (np != want) return fail(OMPRT_ERR_INVALID, "model file: %lld params, want %lld", np, want);
    m->params.resize((size_t)np);
    for (float& v : m->params)
        if (fscanf(fp, "%f", &v) != 1) return fail(OMPRT_ERR_INVALID, "model file: short params");
    return OMPRT_OK;
}

}  // namespace omprt

using namespace omprt;

extern "C" omprt_status omprt_model_load(const char* path) {
    if (!path) {
        std::lock_guard<std::mutex> lk(g_model_mu);
        delete g_model;
    g_pick_cache.clear();
        g_model = nullptr;
        return OMPRT_OK;
    }
    FILE* fp = fopen(path, "r");
    if (!fp) return fail(OMPRT_ERR_INVALID, "cannot open model file %s", path);
    Model* m = new Model();
    const omprt_status st = parse(fp, m);
    fclose(fp);
    if (st != OMPRT_OK) {
        delete m;
        return st;
    }
    std::lock_guard<std::mutex> lk(g_model_mu);
    delete g_model;
    g_pick_cache.clear();
    g_model = m;
    return OMPRT_OK;
}

extern "C" omprt_status omprt_model_features(int64_t n, int32_t dtype, int32_t op, int32_t body,
                                             int64_t chunk, float* h_f16) {
    if (!h_f16) return fail(OMPRT_ERR_INVALID, "output is NULL");
    if (n < 0 || dtype < 0 || dtype >= DT_COUNT_ABI || op < 0 || op > 2 || body < 0 || body > 1)
        return fail(OMPRT_ERR_INVALID, "bad call properties");
    model_features(n, dtype, op, body, chunk, h_f16);
    return OMPRT_OK;
}
