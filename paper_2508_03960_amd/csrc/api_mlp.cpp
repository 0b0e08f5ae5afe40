// C ABI of the learned RF-transition surrogate (include/gbloch.h).
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "consts.hpp"
#include "gbloch.h"
#include "mlp.hpp"
#include "mlp_api.hpp"

using namespace gbs;

namespace {

int mfail(gbs_mlp *m, int code, const std::string &msg) {
    if (m) m->err = msg;
    return code;
}

#define MCHK(expr)                                                                             \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return mfail(m, e_ == hipErrorOutOfMemory ? GBS_E_NOMEM : GBS_E_HIP,               \
                         std::string(#expr) + ": " + hipGetErrorString(e_));                   \
    } while (0)

// Device scratch released on scope exit.
struct Scratch {
    std::vector<void *> ptrs;
    hipError_t get(void **p, size_t n) {
        hipError_t e = hipMalloc(p, n ? n : 256);
        if (e == hipSuccess) ptrs.push_back(*p);
        else *p = nullptr;
        return e;
    }
    ~Scratch() {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t &s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

void default_norm(MlpNorm &n) {
    const double lo[5] = {-1400.0, -100.0, std::log(0.25), std::log(0.03), 0.8};
    const double hi[5] = {1400.0, 100.0, std::log(2.5), std::log(0.3), 1.2};
    for (int k = 0; k < 5; ++k) {
        n.center[k] = (float)(0.5 * (lo[k] + hi[k]));
        n.inv_scale[k] = (float)(2.0 / (hi[k] - lo[k]));
    }
}

int check_tuples(gbs_mlp *m, const void *p, int64_t n) {
    if (!m) return GBS_E_INVALID;
    if (!p) return mfail(m, GBS_E_INVALID, "null device pointer");
    if (n < 0 || n > (int64_t)1 << 31) return mfail(m, GBS_E_INVALID, "tuple count out of range");
    return GBS_OK;
}

// Unit quaternion (w, x, y, z) of a rotation matrix R (row-major), from its
// largest diagonal combination (safe at every angle).
void quaternion_of(const double *R, double q[4]) {
    const double tr = R[0] + R[4] + R[8];
    if (tr >= R[0] && tr >= R[4] && tr >= R[8]) {
        const double w = 0.5 * std::sqrt(1.0 + tr);
        q[0] = w;
        q[1] = (R[7] - R[5]) / (4.0 * w);
        q[2] = (R[2] - R[6]) / (4.0 * w);
        q[3] = (R[3] - R[1]) / (4.0 * w);
    } else if (R[0] >= R[4] && R[0] >= R[8]) {
        const double x = 0.5 * std::sqrt(1.0 + R[0] - R[4] - R[8]);
        q[0] = (R[7] - R[5]) / (4.0 * x);
        q[1] = x;
        q[2] = (R[1] + R[3]) / (4.0 * x);
        q[3] = (R[2] + R[6]) / (4.0 * x);
    } else if (R[4] >= R[8]) {
        const double y = 0.5 * std::sqrt(1.0 - R[0] + R[4] - R[8]);
        q[0] = (R[2] - R[6]) / (4.0 * y);
        q[1] = (R[1] + R[3]) / (4.0 * y);
        q[2] = y;
        q[3] = (R[5] + R[7]) / (4.0 * y);
    } else {
        const double z = 0.5 * std::sqrt(1.0 - R[0] - R[4] + R[8]);
        q[0] = (R[3] - R[1]) / (4.0 * z);
        q[1] = (R[2] + R[6]) / (4.0 * z);
        q[2] = (R[5] + R[7]) / (4.0 * z);
        q[3] = z;
    }
}

// The reference-rotation table of the pulse just set (mlp.hpp): exact
// relaxation-free transitions at B1 scale 1 on the f grid, taken into the
// frame, as angle and axis of their quaternions with continuous signs.
int build_reference(gbs_mlp *m) {
    std::vector<float> tup(5 * (size_t)kRefGrid);
    const double df = 2.0 * kRefFmax / (kRefGrid - 1);
    for (int j = 0; j < kRefGrid; ++j) {
        float *t = tup.data() + 5 * (size_t)j;
        t[0] = (float)(-kRefFmax + j * df);  // a multiple of 1/32 Hz: exact in float
        t[1] = 0.f;
        t[2] = t[3] = INFINITY;
        t[4] = 1.f;
    }
    Scratch s;
    float *d_tup;
    double *d_T;
    MCHK(s.get((void **)&d_tup, sizeof(float) * tup.size()));
    MCHK(s.get((void **)&d_T, sizeof(double) * 12 * (size_t)kRefGrid));
    MCHK(hipMemcpyAsync(d_tup, tup.data(), sizeof(float) * tup.size(), hipMemcpyHostToDevice, m->stream));
    MCHK(mlp_exact_async(m, d_tup, nullptr, kRefGrid, nullptr, d_T, m->stream));
    std::vector<double> T(12 * (size_t)kRefGrid);
    MCHK(hipMemcpyAsync(T.data(), d_T, sizeof(double) * T.size(), hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    std::vector<float4> tab(kRefGrid);
    double prev[4] = {0.0, 0.0, 0.0, 0.0};
    std::vector<std::array<double, 4>> qs(kRefGrid);
    for (int j = 0; j < kRefGrid; ++j) {
        // K = P(-a) A P(-a) with a = -2 pi f tau/2; P(-a) = [[c, s], [-s, c]] in x, y
        const double a = -kTwoPi * (double)tup[5 * (size_t)j] * m->norm.half;
        const double c = std::cos(a), sn = std::sin(a);
        const double *A = T.data() + 12 * (size_t)j;
        const double P[9] = {c, sn, 0.0, -sn, c, 0.0, 0.0, 0.0, 1.0};
        double PA[9], K[9];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k)
                PA[3 * r + k] = P[3 * r] * A[k] + P[3 * r + 1] * A[3 + k] + P[3 * r + 2] * A[6 + k];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k)
                K[3 * r + k] = PA[3 * r] * P[k] + PA[3 * r + 1] * P[3 + k] + PA[3 * r + 2] * P[6 + k];
        double q[4];
        quaternion_of(K, q);
        if (j > 0 && q[0] * prev[0] + q[1] * prev[1] + q[2] * prev[2] + q[3] * prev[3] < 0.0)
            for (double &v : q) v = -v;  // q and -q are the same rotation: keep the path continuous
        for (int i = 0; i < 4; ++i) prev[i] = q[i];
        qs[j] = {q[0], q[1], q[2], q[3]};
    }
    const double sgn = qs[0][0] < 0.0 ? -1.0 : 1.0;
    for (int j = 0; j < kRefGrid; ++j) {
        const double w = sgn * qs[j][0], x = sgn * qs[j][1], y = sgn * qs[j][2], z = sgn * qs[j][3];
        const double v = std::sqrt(x * x + y * y + z * z);
        const double th = 2.0 * std::atan2(v, w);
        tab[j] = v > 1e-300 ? make_float4((float)th, (float)(x / v), (float)(y / v), (float)(z / v))
                            : make_float4((float)th, 0.f, 0.f, 1.f);
    }
    MCHK(hipMemcpy(m->ref, tab.data(), sizeof(float4) * kRefGrid, hipMemcpyHostToDevice));
    m->norm.ref = m->ref;
    return GBS_OK;
}

}  // namespace

namespace gbs {

hipError_t mlp_infer_async(const gbs_mlp *m, const float *tuples, const int32_t *idx, int64_t n, float *T32,
                           hipStream_t st) {
    MlpInferArgs a{tuples, idx, n, (const uint4 *)m->wf, m->w, m->norm, T32};
    return launch_mlp_infer(a, st);
}

hipError_t mlp_infer_rows_async(const gbs_mlp *m, const float *z, const float *df, const float *t1, const float *t2,
                                int64_t n, float4 *rows, int64_t stride, hipStream_t st) {
    MlpInferArgs a{};
    a.N = n;
    a.wf = (const uint4 *)m->wf;
    a.params = m->w;
    a.norm = m->norm;
    a.src_z = z;
    a.src_df = df;
    a.src_t1 = t1;
    a.src_t2 = t2;
    a.fz_per_m = kGammaBar * m->g_ref;
    a.rows = rows;
    a.row_stride = stride;
    return launch_mlp_infer(a, st);
}

hipError_t mlp_exact_async(const gbs_mlp *m, const float *tuples, const int32_t *idx, int64_t n,
                           const int32_t *gate, double *T64, hipStream_t st) {
    MlpExactArgs a{tuples, idx, n, m->wave, (int32_t)m->n_steps, m->dt, m->g_ref, gate, T64};
    return launch_mlp_exact(a, st);
}

}  // namespace gbs

extern "C" {

int gbs_mlp_create(gbs_mlp **out, int device, void *stream, uint64_t seed) {
    if (!out) return GBS_E_INVALID;
    *out = nullptr;
    int nd = 0;
    if (hipGetDeviceCount(&nd) != hipSuccess || device < 0 || device >= nd) return GBS_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return GBS_E_HIP;
    gbs_mlp *m = new (std::nothrow) gbs_mlp();
    if (!m) return GBS_E_NOMEM;
    m->device = device;
    m->stream = (hipStream_t)stream;
    default_norm(m->norm);
    m->norm.half = 0.0;
    const size_t pb = sizeof(float) * kMlpParams;
    if (hipMalloc((void **)&m->w, pb) != hipSuccess || hipMalloc((void **)&m->m, pb) != hipSuccess ||
        hipMalloc((void **)&m->v, pb) != hipSuccess ||
        hipMalloc((void **)&m->wf, sizeof(uint16_t) * 512 * kFragFwd) != hipSuccess ||
        hipMalloc((void **)&m->wb, sizeof(uint16_t) * 512 * kFragBwd) != hipSuccess ||
        hipMalloc((void **)&m->ref, sizeof(float4) * kRefGrid) != hipSuccess) {
        gbs_mlp_destroy(m);
        return GBS_E_NOMEM;
    }
    // PyTorch-style init: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases
    std::vector<float> p(kMlpParams);
    uint64_t s = seed;
    const int offs[9] = {kOffW1, kOffB1, kOffW2, kOffB2, kOffW3, kOffB3, kOffW4, kOffB4, kMlpParams};
    const int fan[8] = {5, 5, 128, 128, 128, 128, 128, 128};
    for (int k = 0; k < 8; ++k) {
        const double bound = 1.0 / std::sqrt((double)fan[k]);
        for (int i = offs[k]; i < offs[k + 1]; ++i) p[i] = (float)((2.0 * uniform01(s) - 1.0) * bound);
    }
    int rc = gbs_mlp_set_params(m, p.data(), kMlpParams);
    if (rc != GBS_OK) {
        gbs_mlp_destroy(m);
        return rc;
    }
    *out = m;
    return GBS_OK;
}

int gbs_mlp_destroy(gbs_mlp *m) {
    if (!m) return GBS_OK;
    (void)hipSetDevice(m->device);
    (void)hipStreamSynchronize(m->stream);
    void *ptrs[] = {m->w, m->m, m->v, m->wf, m->wb, m->wave, m->ref};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete m;
    return GBS_OK;
}

const char *gbs_mlp_last_error(const gbs_mlp *m) { return m ? m->err.c_str() : "null network"; }

int gbs_mlp_set_pulse(gbs_mlp *m, const float *rf_re, const float *rf_im, const float *gx, const float *gy,
                      const float *gz, int64_t n_steps, double dt) {
    if (!m) return GBS_E_INVALID;
    if (!rf_re || !rf_im || !gx || !gy || !gz) return mfail(m, GBS_E_INVALID, "null waveform");
    if (n_steps < 1 || n_steps > (1 << 24)) return mfail(m, GBS_E_INVALID, "n_steps out of range");
    if (!(dt > 0.0) || !std::isfinite(dt)) return mfail(m, GBS_E_INVALID, "dt must be positive");
    double g_ref = 0.0;
    for (int64_t i = 0; i < n_steps; ++i) {
        if (gx[i] != 0.f || gy[i] != 0.f) return mfail(m, GBS_E_INVALID, "pulse must be Gz-only (gx = gy = 0)");
        if (!std::isfinite(rf_re[i]) || !std::isfinite(rf_im[i]) || !std::isfinite(gz[i]))
            return mfail(m, GBS_E_INVALID, "non-finite waveform");
        g_ref = std::max(g_ref, (double)std::fabs(gz[i]));
    }
    if (g_ref == 0.0) return mfail(m, GBS_E_INVALID, "pulse has no slice gradient (gz all zero)");
    MCHK(hipSetDevice(m->device));
    m->has_pulse = false;
    std::vector<float4> w(n_steps);
    for (int64_t i = 0; i < n_steps; ++i) w[i] = make_float4(rf_re[i], rf_im[i], gz[i], 0.f);
    if (m->wave) {
        (void)hipStreamSynchronize(m->stream);
        (void)hipFree(m->wave);
        m->wave = nullptr;
    }
    MCHK(hipMalloc((void **)&m->wave, sizeof(float4) * n_steps));
    MCHK(hipMemcpy(m->wave, w.data(), sizeof(float4) * n_steps, hipMemcpyHostToDevice));
    m->rf_re.assign(rf_re, rf_re + n_steps);
    m->rf_im.assign(rf_im, rf_im + n_steps);
    m->gz.assign(gz, gz + n_steps);
    m->n_steps = n_steps;
    m->dt = dt;
    m->g_ref = g_ref;
    m->norm.half = 0.5 * (double)n_steps * dt;
    if (int rc = build_reference(m)) return rc;
    m->has_pulse = true;
    return GBS_OK;
}

int gbs_mlp_set_norm(gbs_mlp *m, const float center[5], const float scale[5]) {
    if (!m) return GBS_E_INVALID;
    if (!center || !scale) return mfail(m, GBS_E_INVALID, "null normalization");
    for (int k = 0; k < 5; ++k) {
        if (!(scale[k] != 0.f) || !std::isfinite(scale[k]) || !std::isfinite(center[k]))
            return mfail(m, GBS_E_INVALID, "normalization must be finite with scale != 0");
    }
    for (int k = 0; k < 5; ++k) {
        m->norm.center[k] = center[k];
        m->norm.inv_scale[k] = 1.f / scale[k];
    }
    return GBS_OK;
}

int gbs_mlp_get_params(gbs_mlp *m, float *params, int64_t n) {
    if (!m) return GBS_E_INVALID;
    if (!params || n != kMlpParams) return mfail(m, GBS_E_INVALID, "params must be float[GBS_MLP_PARAMS]");
    MCHK(hipSetDevice(m->device));
    MCHK(hipStreamSynchronize(m->stream));
    MCHK(hipMemcpy(params, m->w, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    return GBS_OK;
}

int gbs_mlp_set_params(gbs_mlp *m, const float *params, int64_t n) {
    if (!m) return GBS_E_INVALID;
    if (!params || n != kMlpParams) return mfail(m, GBS_E_INVALID, "params must be float[GBS_MLP_PARAMS]");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(params[i])) return mfail(m, GBS_E_INVALID, "non-finite parameter");
    MCHK(hipSetDevice(m->device));
    MCHK(hipStreamSynchronize(m->stream));
    MCHK(hipMemcpy(m->w, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    MCHK(launch_fill_f32(m->m, kMlpParams, 0.f, m->stream));
    MCHK(launch_fill_f32(m->v, kMlpParams, 0.f, m->stream));
    // padding positions of the fragments stay zero; every weight is written by the pack
    MCHK(launch_fill_f32((float *)m->wf, 256 * kFragFwd, 0.f, m->stream));
    MCHK(launch_fill_f32((float *)m->wb, 256 * kFragBwd, 0.f, m->stream));
    MCHK(launch_mlp_pack(m->w, m->wf, m->wb, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    m->t = 0;
    return GBS_OK;
}

int gbs_mlp_exact(gbs_mlp *m, const float *tuples, int64_t n, double *T) {
    int rc = check_tuples(m, tuples, n);
    if (rc != GBS_OK) return rc;
    if (!T) return mfail(m, GBS_E_INVALID, "null output");
    if (!m->has_pulse) return mfail(m, GBS_E_STATE, "no pulse set");
    MCHK(hipSetDevice(m->device));
    MCHK(mlp_exact_async(m, tuples, nullptr, n, nullptr, T, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return GBS_OK;
}

int gbs_mlp_infer(gbs_mlp *m, const float *tuples, int64_t n, float *T) {
    int rc = check_tuples(m, tuples, n);
    if (rc != GBS_OK) return rc;
    if (!T) return mfail(m, GBS_E_INVALID, "null output");
    if (!m->has_pulse) return mfail(m, GBS_E_STATE, "no pulse set");
    MCHK(hipSetDevice(m->device));
    MCHK(mlp_infer_async(m, tuples, nullptr, n, T, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return GBS_OK;
}

namespace {

struct TrainBufs {
    Scratch s;
    uint16_t *act_h, *act_l, *dz_h, *dz_l;
    float *K;
    hipError_t alloc(int64_t n, int B) {
        hipError_t e;
        if ((e = s.get((void **)&act_h, sizeof(uint16_t) * kActRows * (size_t)B)) != hipSuccess) return e;
        if ((e = s.get((void **)&act_l, sizeof(uint16_t) * kActRows * (size_t)B)) != hipSuccess) return e;
        if ((e = s.get((void **)&dz_h, sizeof(uint16_t) * kDzRows * (size_t)B)) != hipSuccess) return e;
        if ((e = s.get((void **)&dz_l, sizeof(uint16_t) * kDzRows * (size_t)B)) != hipSuccess) return e;
        return s.get((void **)&K, sizeof(float) * 12 * (size_t)n);
    }
    MlpGradAdamArgs grad_args(int32_t B) const {
        MlpGradAdamArgs g{};
        g.act_h = act_h;
        g.act_l = act_l;
        g.dz_h = dz_h;
        g.dz_l = dz_l;
        g.B = B;
        return g;
    }
    MlpTrainArgs train_args(const gbs_mlp *m, const float *tuples, int64_t n, int B, float *loss) const {
        MlpTrainArgs a{};
        a.tuples = tuples;
        a.targets = K;
        a.N = n;
        a.pa = 1;
        a.pc = 0;
        a.j0 = 0;
        a.B = B;
        a.wf = (const uint4 *)m->wf;
        a.wb = (const uint4 *)m->wb;
        a.params = m->w;
        a.norm = m->norm;
        a.act_h = act_h;
        a.act_l = act_l;
        a.dz_h = dz_h;
        a.dz_l = dz_l;
        a.loss = loss;
        return a;
    }
};

}  // namespace

int gbs_mlp_loss_grad(gbs_mlp *m, const float *tuples, const double *T_exact, int64_t n, float *grad, float *loss) {
    int rc = check_tuples(m, tuples, n);
    if (rc != GBS_OK) return rc;
    if (!T_exact || !grad || !loss) return mfail(m, GBS_E_INVALID, "null argument");
    if (n < 64 || n % 64 || n > (1 << 20)) return mfail(m, GBS_E_INVALID, "n must be a multiple of 64 in [64, 2^20]");
    if (!m->has_pulse) return mfail(m, GBS_E_STATE, "no pulse set (the target frame needs its duration)");
    MCHK(hipSetDevice(m->device));
    TrainBufs tb;
    MCHK(tb.alloc(n, (int)n));
    float *dloss;
    MCHK(tb.s.get((void **)&dloss, sizeof(float)));
    MCHK(launch_fill_f32(dloss, 1, 0.f, m->stream));
    MCHK(launch_mlp_targets(tuples, T_exact, n, m->norm, tb.K, m->stream));
    MCHK(launch_mlp_train_fb(tb.train_args(m, tuples, n, (int)n, dloss), m->stream));
    MlpGradAdamArgs ga = tb.grad_args((int32_t)n);
    ga.grad_out = grad;
    MCHK(launch_mlp_grad_adam(ga, m->stream));
    MCHK(hipMemcpyAsync(loss, dloss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return GBS_OK;
}

int gbs_mlp_train(gbs_mlp *m, const float *tuples, const double *T_exact, int64_t n, const gbs_train_cfg *cfg,
                  float *loss_hist, int64_t hist_len) {
    int rc = check_tuples(m, tuples, n);
    if (rc != GBS_OK) return rc;
    if (!T_exact || !cfg) return mfail(m, GBS_E_INVALID, "null argument");
    if (cfg->batch < 256 || cfg->batch % 256 || cfg->batch > (1 << 20))
        return mfail(m, GBS_E_INVALID, "batch must be a multiple of 256 in [256, 2^20]");
    if (n < cfg->batch) return mfail(m, GBS_E_INVALID, "fewer samples than one batch");
    if (cfg->epochs < 1) return mfail(m, GBS_E_INVALID, "epochs must be >= 1");
    if (!(cfg->lr_max > 0.f) || !(cfg->lr_min >= 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) ||
        !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) || !(cfg->eps > 0.f))
        return mfail(m, GBS_E_INVALID, "bad optimizer settings");
    if (!m->has_pulse) return mfail(m, GBS_E_STATE, "no pulse set (the target frame needs its duration)");
    MCHK(hipSetDevice(m->device));
    const int B = cfg->batch;
    const int64_t per_epoch = n / B, total = per_epoch * cfg->epochs;
    TrainBufs tb;
    MCHK(tb.alloc(n, B));
    float *dloss;
    MCHK(tb.s.get((void **)&dloss, sizeof(float) * total));
    MCHK(launch_fill_f32(dloss, total, 0.f, m->stream));
    MCHK(launch_mlp_targets(tuples, T_exact, n, m->norm, tb.K, m->stream));
    uint64_t rs = cfg->seed;
    int64_t k = 0;
    for (int e = 0; e < cfg->epochs; ++e) {
        // sample order of this epoch: j -> (pa j + pc) mod n with gcd(pa, n) = 1
        uint64_t pa = 1;
        for (int tries = 0; tries < 64; ++tries) {
            const uint64_t c = 1 + splitmix64(rs) % (uint64_t)(n > 1 ? n - 1 : 1);
            if (std::gcd(c, (uint64_t)n) == 1) {
                pa = c;
                break;
            }
        }
        const uint64_t pc = splitmix64(rs) % (uint64_t)n;
        for (int64_t b = 0; b < per_epoch; ++b, ++k) {
            MlpTrainArgs a = tb.train_args(m, tuples, n, B, dloss + k);
            a.pa = pa;
            a.pc = pc;
            a.j0 = b * B;
            MCHK(launch_mlp_train_fb(a, m->stream));
            m->t += 1;
            const double frac = (double)k / (double)total;  // first step at lr_max
            const double lr = cfg->lr_min + 0.5 * (cfg->lr_max - cfg->lr_min) * (1.0 + std::cos(kTwoPi * 0.5 * frac));
            MlpGradAdamArgs ad = tb.grad_args(B);
            ad.w = m->w;
            ad.m = m->m;
            ad.v = m->v;
            ad.wf = m->wf;
            ad.wb = m->wb;
            ad.lr = (float)lr;
            ad.beta1 = cfg->beta1;
            ad.beta2 = cfg->beta2;
            ad.eps = cfg->eps;
            ad.corr1 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta1, (double)m->t)));
            ad.corr2 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta2, (double)m->t)));
            ad.grad_out = nullptr;
            MCHK(launch_mlp_grad_adam(ad, m->stream));
        }
    }
    if (loss_hist && hist_len > 0) {
        const int64_t nh = std::min(hist_len, total);
        MCHK(hipMemcpyAsync(loss_hist, dloss, sizeof(float) * nh, hipMemcpyDeviceToHost, m->stream));
    }
    MCHK(hipStreamSynchronize(m->stream));
    return GBS_OK;
}

}  // extern "C"
