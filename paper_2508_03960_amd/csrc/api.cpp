// C ABI of the grouped-isochromat Bloch simulator (include/gbloch.h).
//
// The context owns: a device copy of the sequence waveform, after
// gbs_build_groups a group-sorted copy of the phantom (sorted by the x-group
// key, so every x-group is one contiguous run) with per-axis group ids and
// group tables, and the small device arrays of each mode's schedule (job
// descriptors, per-sample tables), built by the setters.  Everything a
// simulation writes besides its outputs (the magnetization state in layout
// order, combined-transition and map tables, group sums, partial sums, the
// FP64 state and the transition cache of the conventional method) lives in
// the caller's workspace; gbs_simulate allocates nothing.  The caller owns
// the phantom arrays, the workspace and the outputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_set>
#include <vector>

#include "adc.hpp"
#include "adj.hpp"
#include "cached.hpp"
#include "consts.hpp"
#include "gbloch.h"
#include "groups.hpp"
#include "kernels.hpp"
#include "mlp.hpp"
#include "mlp_api.hpp"
#include "noalloc.hpp"
#include "pairs.hpp"
#include "plain_coils.hpp"
#include "plan.hpp"

using namespace gbs;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n) {
        if (n == 0) n = 256;
        if (p && n <= cap) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, n);
        if (e == hipSuccess) cap = n;
        else p = nullptr;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <class T>
    T *as() const {
        return (T *)p;
    }
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Regions of a caller's workspace, carved in order.  The first 256 bytes are
// never handed out, so a zero workspace offset stored in a job descriptor
// means "no table".
struct WsCarve {
    size_t off = 256;
    size_t take(size_t bytes) {
        const size_t o = off;
        off = align256(off + (bytes ? bytes : 1));
        return o;
    }
};

// A workspace-relative address: job descriptors are assembled with workspace
// offsets in their table and sum pointers, and the offsets are turned into
// device addresses once the workspace is known (relocate_jobs).
template <class T>
T *ws_rel(size_t off) {
    return reinterpret_cast<T *>(static_cast<uintptr_t>(off));
}

// Record, for n consecutive structs of type T at byte offset arr in img, the
// byte offsets of the given pointer fields that hold a workspace offset.
template <class T>
void add_relocs(std::vector<size_t> &slots, const std::vector<char> &img, size_t arr, size_t n,
                std::initializer_list<size_t> fields) {
    for (size_t i = 0; i < n; ++i)
        for (size_t f : fields) {
            const size_t at = arr + i * sizeof(T) + f;
            uintptr_t v = 0;
            std::memcpy(&v, img.data() + at, sizeof(v));
            if (v) slots.push_back(at);
        }
}

// Everything about a grouped simulation that depends only on the sequence and
// the groups: the pass schedule, the arena layout, the per-sample tables and
// the job arrays (uploaded once).  Rebuilt after set_sequence/build_groups.
struct GroupedPlan {
    bool valid = false;
    Plan plan;
    // workspace layout: state in layout order (mx, my, mz planes of Kpad
    // floats, then the final (mx, my, mz, 0) rows), table arena, group sums,
    // partial sums of stepped blocks, surrogate buffers
    size_t w_state = 0, w_tabs = 0, w_gsum = 0, w_partial = 0, w_surr = 0, ws_bytes = 0;
    // job image slots that hold workspace offsets, and the workspace the
    // device copy of the jobs was relocated for (null: not uploaded)
    std::vector<size_t> relocs;
    const void *uploaded_ws = nullptr;
    bool zbuilt = false;
    std::vector<size_t> rf_off, gsum_off;
    // no-grads transitions composed per tissue group: (composed rows, x-group rows)
    std::vector<std::pair<size_t, size_t>> expand;
    // Gx+Gz transitions composed per two-axis group: (arena offset, RF job)
    std::vector<std::pair<size_t, int>> pair_jobs;
    size_t gsum_count = 0;
    int64_t max_rf_groups = 0, max_tab = 0;
    int max_adc_groups = 0, max_adc_samples = 0;
    int n_rf = 0, n_fold = 0, n_tab = 0, n_adc = 0, n_adclin = 0, max_adclin_groups = 0;
    int64_t max_fold_groups = 0;
    size_t o_rf = 0, o_fold = 0, o_tab = 0, o_adc = 0, o_adclin = 0, o_sweep = 0;
    // execution: runs of grouped ops fused into sweeps, plain steps between
    struct Seg {
        int op_begin, op_end, need;
        bool write_m;
        double bytes_per_iso, flops_per_iso;
        int n_head = 0;  // kEmitHead: general ops before the emission run
    };
    std::vector<Seg> segs;
    std::vector<std::pair<int, int>> exec;  // (0, segment) or (1, index into plan.ops)
    // kPartials segments: their reduction jobs [first, first + count) at o_part
    std::vector<std::pair<int, int>> seg_parts;
    size_t o_part = 0, w_part = 0;
    int64_t n_ops = 0;
    // learned surrogate for one distinct RF transition (surr_rf >= 0); the
    // RF jobs at o_rf_surr skip its exact composition.  s_* are offsets in
    // the workspace's surrogate region.
    int surr_rf = -1;
    int64_t surr_groups = 0;
    int surr_n_check = 0;
    size_t o_rf_surr = 0;
    size_t s_tuples = 0, s_T32 = 0, s_exact = 0, s_res = 0, s_fb = 0;
};

}  // namespace

struct gbs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // phantom (caller-owned views, natural order)
    int64_t K = 0;
    PhantomPtrs ph{};
    bool has_ph = false;
    // sequence
    HostSeq seq;
    bool has_seq = false;
    std::vector<BlockClass> cls;
    DevBuf d_wave, d_adc;
    // groups and the group-sorted copy
    uint32_t axes = 0;
    bool groups_valid = false;
    int64_t ng[3] = {-1, -1, -1};
    int64_t Kint = 0;  // isochromats in the padded group-sorted layout (multiple of 8)
    int64_t Kpad = 0;
    DevBuf perm, inv, xi, yi, zi, t1i, t2i, dfi, m0i, gid[3], gtab[3], gcount[3];
    DevBuf xstart;  // first layout slot of every x-group, and Kint after the last
    // no-grads groups (GBS_AX_N): (0, T1, T2, df) per group, and the group of each x-group
    int64_t n_tissue = -1;
    DevBuf ttab, tmap;
    // two-axis groups (GBS_AX_XZ): the layout's runs of equal (x-group,
    // z-group); run of every 4-slot quad, and (x, T1, T2, df), z per run
    int64_t n_runs = -1;
    DevBuf run_of4, rtab, rz;
    // receive coils (gbs_set_coils; caller-owned views [n_coils][K] in natural
    // order) and their group-sorted copy (planes re, im per coil, Kpad each)
    int32_t n_coils = 1;
    const float *coil_re = nullptr, *coil_im = nullptr;
    DevBuf coil_l;
    bool coil_l_valid = false;
    // grouped schedule on the device: job descriptors (relocated to the
    // workspace of the call) and per-sample tables; validation flag
    DevBuf jobs, samp, flag;
    std::vector<char> host_jobs, patched_jobs;
    std::vector<double2> host_samp;
    double2 *partial = nullptr;  // per-workgroup sample sums of the current call (workspace)
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    // second stream of the context (default priority): the copy of the final
    // state into the caller's order runs on it beside the ADC evaluation
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    std::vector<hipEvent_t> pev;  // GBS_PROFILE: one (start, stop) pair per pass launch
    GroupedPlan gp;
    // learned surrogate (not owned)
    gbs_mlp *mlp = nullptr;
    float surr_tol = 1e-3f;
    int32_t surr_check = 32;
    uint64_t surr_seed = 0;
    DevBuf surr_idx;  // seeded spot-check groups
    // GBS_CACHED with the surrogate: the cache entry it fills (-1: none) and
    // its seeded spot-check isochromats
    int csurr_entry = -1;
    int32_t csurr_n_check = 0;
    DevBuf csurr_idx;
    // gradient of the signal (adjoint): flattened ops, checkpoints, partials
    DevBuf adj_ops, adj_samp, adj_ckpt, adj_sub, adj_sig, adj_grf, adj_gt;
    AdjArgs adj{};
    bool adj_ready = false;
    bool pplan_valid = false;
    Plan pplan;  // plain schedule
    // conventional method with per-isochromat transition caching (GBS_CACHED):
    // schedule, per-sample tables of its direct ADC operations (row offset per
    // operation) and, with GBS_PROFILE, the kind of each timed launch.  The
    // cache itself (3 float4 rows of K per entry) is in the workspace.
    bool cplan_valid = false;
    Plan cplan;
    std::vector<int64_t> csamp_off;
    DevBuf csamp;
    std::vector<int> cprof_kind;
};

static int fail(gbs_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

int gbs::ctx_device(const gbs_ctx *ctx) { return ctx ? ctx->device : -1; }
int gbs::ctx_fail(gbs_ctx *ctx, int code, const char *msg) { return fail(ctx, code, msg); }

static int refresh_plans(gbs_ctx *ctx);
static int build_coil_layout(gbs_ctx *ctx);
static int build_grouped_plan(gbs_ctx *ctx);

#define HIPCHK(expr)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(ctx, e_ == hipErrorOutOfMemory ? GBS_E_NOMEM : GBS_E_HIP,              \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                    \
    } while (0)

#define ALLOC(buf, bytes)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (buf).ensure(bytes);                                                   \
        if (e_ != hipSuccess)                                                                  \
            return fail(ctx, GBS_E_NOMEM, std::string("device allocation of ") +               \
                                              std::to_string((size_t)(bytes)) + " bytes failed"); \
    } while (0)

static const char *status_text(int s) {
    switch (s) {
        case GBS_OK: return "ok";
        case GBS_E_INVALID: return "invalid argument";
        case GBS_E_STATE: return "invalid call order or stale state";
        case GBS_E_HIP: return "HIP runtime error";
        case GBS_E_NOMEM: return "out of memory";
        case GBS_E_WORKSPACE: return "workspace missing, too small or misaligned";
        default: return "unknown status";
    }
}

extern "C" {

const char *gbs_strerror(int status) { return status_text(status); }

const char *gbs_last_error(const gbs_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int gbs_create(gbs_ctx **out, int device, void *stream) {
    if (!out) return GBS_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return GBS_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return GBS_E_HIP;
    if (noalloc_setup(device) != hipSuccess) return GBS_E_HIP;  // this device's static scratch (gbs_simulate_static)
    gbs_ctx *ctx = new (std::nothrow) gbs_ctx();
    if (!ctx) return GBS_E_NOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)stream;
    for (auto &e : ctx->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            gbs_destroy(ctx);
            return GBS_E_HIP;
        }
    }
    if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming) != hipSuccess) {
        gbs_destroy(ctx);
        return GBS_E_HIP;
    }
    *out = ctx;
    return GBS_OK;
}

int gbs_destroy(gbs_ctx *ctx) {
    if (!ctx) return GBS_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);  // a failed call may have left work there
    DevBuf *bufs[] = {&ctx->d_wave, &ctx->d_adc, &ctx->perm, &ctx->inv, &ctx->xi, &ctx->yi, &ctx->zi, &ctx->t1i,
                      &ctx->t2i, &ctx->dfi, &ctx->m0i, &ctx->jobs, &ctx->samp, &ctx->flag, &ctx->surr_idx, &ctx->csurr_idx,
                      &ctx->adj_ops, &ctx->adj_samp, &ctx->adj_ckpt, &ctx->adj_sub, &ctx->adj_sig, &ctx->adj_grf,
                      &ctx->adj_gt, &ctx->csamp, &ctx->ttab, &ctx->tmap, &ctx->coil_l, &ctx->run_of4, &ctx->xstart,
                      &ctx->rtab, &ctx->rz};
    for (DevBuf *b : bufs) b->release();
    for (int a = 0; a < 3; ++a) {
        ctx->gid[a].release();
        ctx->gtab[a].release();
        ctx->gcount[a].release();
    }
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : ctx->pev) (void)hipEventDestroy(e);
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->join) (void)hipEventDestroy(ctx->join);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    delete ctx;
    return GBS_OK;
}

int gbs_set_phantom(gbs_ctx *ctx, int64_t K, const float *x, const float *y, const float *z,
                    const float *t1, const float *t2, const float *df_hz, const float *m0) {
    if (!ctx) return GBS_E_INVALID;
    if (K <= 0 || K > (int64_t)INT32_MAX - 4096)
        return fail(ctx, GBS_E_INVALID, "K must be in [1, 2^31 - 4096]");
    if (!x || !y || !z || !t1 || !t2 || !df_hz || !m0) return fail(ctx, GBS_E_INVALID, "null phantom array");
    HIPCHK(hipSetDevice(ctx->device));
    ctx->has_ph = false;
    ctx->groups_valid = false;
    ctx->gp.valid = false;
    ctx->adj_ready = false;
    ctx->n_coils = 1;  // sensitivities belong to the previous phantom
    ctx->coil_re = ctx->coil_im = nullptr;
    ctx->coil_l_valid = false;
    PhantomPtrs ph{x, y, z, t1, t2, df_hz, m0};
    ALLOC(ctx->flag, 256);
    HIPCHK(launch_fill_f64(ctx->flag.as<double>(), 1, ctx->stream));
    HIPCHK(launch_validate_phantom(K, ph, ctx->flag.as<int>(), ctx->stream));
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, ctx->flag.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (bad) return fail(ctx, GBS_E_INVALID, "phantom has NaN/inf values or T1/T2 <= 0");
    ctx->K = K;
    ctx->ph = ph;
    ctx->has_ph = true;
    return refresh_plans(ctx);  // one coil again: stepped launches take 256 samples
}

int gbs_set_coils(gbs_ctx *ctx, int32_t n_coils, const float *sens_re, const float *sens_im) {
    if (!ctx) return GBS_E_INVALID;
    if (!ctx->has_ph) return fail(ctx, GBS_E_STATE, "gbs_set_coils before gbs_set_phantom");
    if (n_coils < 1 || n_coils > GBS_MAX_COILS)
        return fail(ctx, GBS_E_INVALID, "n_coils must be in [1, " + std::to_string(GBS_MAX_COILS) + "]");
    if (!sens_re != !sens_im) return fail(ctx, GBS_E_INVALID, "sens_re and sens_im must both be set or both null");
    if (!sens_re && n_coils != 1) return fail(ctx, GBS_E_INVALID, "null sensitivities need n_coils = 1");
    HIPCHK(hipSetDevice(ctx->device));
    if (sens_re) {
        ALLOC(ctx->flag, 256);
        HIPCHK(launch_fill_f64(ctx->flag.as<double>(), 1, ctx->stream));
        const int64_t n = (int64_t)n_coils * ctx->K;
        HIPCHK(launch_check_finite(n, sens_re, ctx->flag.as<int>(), ctx->stream));
        HIPCHK(launch_check_finite(n, sens_im, ctx->flag.as<int>(), ctx->stream));
        int bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, ctx->flag.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (bad) return fail(ctx, GBS_E_INVALID, "coil sensitivities have NaN/inf values");
    }
    ctx->n_coils = n_coils;
    ctx->coil_re = sens_re;
    ctx->coil_im = sens_im;
    ctx->coil_l_valid = false;
    return refresh_plans(ctx);  // stepped launches are cut to 256 / n_coils samples
}

int gbs_set_sequence(gbs_ctx *ctx, const gbs_block *blocks, int64_t n_blocks, const float *rf_re,
                     const float *rf_im, const float *gx, const float *gy, const float *gz,
                     int64_t total_steps, const int32_t *adc_idx, int64_t total_samples, double dt) {
    if (!ctx) return GBS_E_INVALID;
    std::string err;
    int rc = validate_sequence(blocks, n_blocks, total_steps, adc_idx, total_samples, dt, err);
    if (rc != GBS_OK) return fail(ctx, rc, err);
    if (total_steps > 0 && (!rf_re || !rf_im || !gx || !gy || !gz))
        return fail(ctx, GBS_E_INVALID, "null waveform array");
    for (int64_t j = 0; j < total_steps; ++j)
        if (!std::isfinite(rf_re[j]) || !std::isfinite(rf_im[j]) || !std::isfinite(gx[j]) ||
            !std::isfinite(gy[j]) || !std::isfinite(gz[j]))
            return fail(ctx, GBS_E_INVALID, "non-finite waveform sample at step " + std::to_string(j));
    HIPCHK(hipSetDevice(ctx->device));
    ctx->has_seq = false;
    ctx->gp.valid = false;
    ctx->pplan_valid = false;
    ctx->cplan_valid = false;
    ctx->adj_ready = false;
    copy_sequence(ctx->seq, blocks, n_blocks, rf_re, rf_im, gx, gy, gz, total_steps, adc_idx, total_samples, dt);
    ctx->cls = classify(ctx->seq);
    std::vector<StepW> w((size_t)total_steps);
    for (int64_t j = 0; j < total_steps; ++j) {
        const double re = rf_re[j], im = rf_im[j];
        w[j] = StepW{rf_re[j], rf_im[j], (float)(re * re + im * im), gx[j], gy[j], gz[j], 0.f, 0.f};
    }
    ALLOC(ctx->d_wave, sizeof(StepW) * (size_t)total_steps);
    ALLOC(ctx->d_adc, sizeof(int32_t) * (size_t)total_samples);
    if (total_steps)
        HIPCHK(hipMemcpy(ctx->d_wave.p, w.data(), sizeof(StepW) * (size_t)total_steps, hipMemcpyHostToDevice));
    if (total_samples)
        HIPCHK(hipMemcpy(ctx->d_adc.p, adc_idx, sizeof(int32_t) * (size_t)total_samples, hipMemcpyHostToDevice));
    ctx->has_seq = true;
    return refresh_plans(ctx);
}

int gbs_build_groups(gbs_ctx *ctx, uint32_t axes) {
    if (!ctx) return GBS_E_INVALID;
    if (!ctx->has_ph) return fail(ctx, GBS_E_STATE, "gbs_build_groups before gbs_set_phantom");
    if (!(axes & GBS_AX_X) || (axes & ~31u))
        return fail(ctx, GBS_E_INVALID, "axes must include GBS_AX_X and only X|Y|Z|N|XZ");
    if ((axes & GBS_AX_XZ) && !(axes & GBS_AX_Z))
        return fail(ctx, GBS_E_INVALID, "GBS_AX_XZ needs GBS_AX_Z");
    HIPCHK(hipSetDevice(ctx->device));
    ctx->groups_valid = false;
    ctx->gp.valid = false;
    ctx->coil_l_valid = false;
    const int64_t K = ctx->K;
    const int64_t cap = (8 * K + 1023) / 1024 * 1024;  // padded layout is at most 8 K long
    const size_t scratch_bytes = group_scratch_bytes(K) + 4096;
    DevBuf scratch, gid_nat[3], order, perm_tmp, src_tmp;
    auto cleanup = [&]() {
        scratch.release();
        for (auto &g : gid_nat) g.release();
        order.release();
        perm_tmp.release();
        src_tmp.release();
    };
    auto fail_hip = [&](hipError_t e, const char *what) {
        cleanup();
        return fail(ctx, e == hipErrorOutOfMemory ? GBS_E_NOMEM : GBS_E_HIP,
                    std::string(what) + ": " + hipGetErrorString(e));
    };
    if (scratch.ensure(scratch_bytes) != hipSuccess || order.ensure(4 * K) != hipSuccess ||
        perm_tmp.ensure(4 * cap) != hipSuccess || src_tmp.ensure(4 * cap) != hipSuccess) {
        cleanup();
        return fail(ctx, GBS_E_NOMEM, "grouping scratch allocation failed");
    }
    // 1. group every requested axis by its key (r_a, T1, T2, dB0)
    const float *coord[3] = {ctx->ph.x, ctx->ph.y, ctx->ph.z};
    for (int a = 0; a < 3; ++a) {
        ctx->ng[a] = -1;
        if (!(axes & (1u << a))) {
            ctx->gid[a].release();
            ctx->gtab[a].release();
            ctx->gcount[a].release();
            continue;
        }
        if (gid_nat[a].ensure(4 * K) != hipSuccess) {
            cleanup();
            return fail(ctx, GBS_E_NOMEM, "grouping scratch allocation failed");
        }
        ALLOC(ctx->gtab[a], sizeof(float4) * K);
        ALLOC(ctx->gcount[a], sizeof(int32_t) * K);
        int64_t G = 0;
        hipError_t e = group_axis(K, coord[a], ctx->ph.t1, ctx->ph.t2, ctx->ph.df, scratch.p, scratch_bytes,
                                  gid_nat[a].as<int32_t>(), ctx->gtab[a].as<float4>(), ctx->gcount[a].as<int32_t>(),
                                  order.as<int32_t>(), &G, ctx->stream);
        if (e != hipSuccess) return fail_hip(e, "grouping failed");
        ctx->ng[a] = G;
    }
    // no-grads groups: the distinct (T1, T2, dB0) of the x-group keys, each x
    // group mapped to its own (every x-group key contains exactly one)
    ctx->n_tissue = -1;
    if (axes & GBS_AX_N) {
        const int64_t Gx = ctx->ng[0];
        std::vector<float4> xt((size_t)Gx);
        HIPCHK(hipMemcpyAsync(xt.data(), ctx->gtab[0].p, sizeof(float4) * (size_t)Gx, hipMemcpyDeviceToHost,
                              ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        auto canon = [](float v) { return v == 0.0f ? 0.0f : v; };  // -0 == +0
        std::vector<std::array<float, 3>> keys((size_t)Gx);
        for (int64_t g = 0; g < Gx; ++g) keys[g] = {canon(xt[g].y), canon(xt[g].z), canon(xt[g].w)};
        std::vector<std::array<float, 3>> uniq(keys);
        std::sort(uniq.begin(), uniq.end());
        uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
        std::vector<int32_t> map((size_t)Gx);
        for (int64_t g = 0; g < Gx; ++g)
            map[g] = (int32_t)(std::lower_bound(uniq.begin(), uniq.end(), keys[g]) - uniq.begin());
        std::vector<float4> tt(uniq.size());
        for (size_t i = 0; i < uniq.size(); ++i) tt[i] = make_float4(0.0f, uniq[i][0], uniq[i][1], uniq[i][2]);
        ALLOC(ctx->ttab, sizeof(float4) * tt.size());
        ALLOC(ctx->tmap, sizeof(int32_t) * map.size());
        HIPCHK(hipMemcpy(ctx->ttab.p, tt.data(), sizeof(float4) * tt.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(ctx->tmap.p, map.data(), sizeof(int32_t) * map.size(), hipMemcpyHostToDevice));
        ctx->n_tissue = (int64_t)uniq.size();
    } else {
        ctx->ttab.release();
        ctx->tmap.release();
    }
    // 2. the padded group-sorted layout: (x-group, z-group) runs of multiples of 8
    int64_t kint = 0;
    hipError_t e = build_layout(K, gid_nat[0].as<int32_t>(), (axes & GBS_AX_Z) ? gid_nat[2].as<int32_t>() : nullptr,
                                scratch.p, scratch_bytes, perm_tmp.as<int32_t>(), src_tmp.as<int32_t>(), cap, &kint,
                                ctx->stream);
    if (e != hipSuccess) return fail_hip(e, "layout failed");
    const int64_t Kpad = (kint + 1023) / 1024 * 1024;
    ALLOC(ctx->perm, 4 * Kpad);
    HIPCHK(hipMemcpyAsync(ctx->perm.p, perm_tmp.p, 4 * Kpad, hipMemcpyDeviceToDevice, ctx->stream));
    ALLOC(ctx->inv, 4 * K);
    HIPCHK(launch_invert(Kpad, ctx->perm.as<int32_t>(), ctx->inv.as<int32_t>(), ctx->stream));
    const int32_t *src = src_tmp.as<int32_t>();
    for (int a = 0; a < 3; ++a) {
        if (!(axes & (1u << a))) continue;
        ALLOC(ctx->gid[a], sizeof(int32_t) * Kpad);
        HIPCHK(launch_gather_i32(Kpad, Kpad, src, gid_nat[a].as<int32_t>(), ctx->gid[a].as<int32_t>(), ctx->stream));
    }
    ALLOC(ctx->xstart, sizeof(int32_t) * (size_t)(ctx->ng[0] + 1));
    HIPCHK(launch_group_starts(kint, ctx->gid[0].as<int32_t>(), ctx->ng[0], ctx->xstart.as<int32_t>(), ctx->stream));
    DevBuf *dst[7] = {&ctx->xi, &ctx->yi, &ctx->zi, &ctx->t1i, &ctx->t2i, &ctx->dfi, &ctx->m0i};
    const float *from[7] = {ctx->ph.x, ctx->ph.y, ctx->ph.z, ctx->ph.t1, ctx->ph.t2, ctx->ph.df, ctx->ph.m0};
    for (int i = 0; i < 7; ++i) {
        ALLOC(*dst[i], 4 * Kpad);
        HIPCHK(launch_gather_f32(Kpad, Kpad, src, from[i], dst[i]->as<float>(), ctx->stream));
    }
    HIPCHK(launch_zero_padding(Kpad, ctx->perm.as<int32_t>(), ctx->m0i.as<float>(), ctx->stream));
    // two-axis groups: the runs of equal (x-group, z-group) in the layout
    ctx->n_runs = -1;
    if (axes & GBS_AX_XZ) {
        const int64_t n4 = kint / 4;
        DevBuf flags;
        if (flags.ensure((size_t)n4) != hipSuccess) {
            cleanup();
            return fail(ctx, GBS_E_NOMEM, "run flag allocation failed");
        }
        HIPCHK(launch_run_flags(n4, ctx->gid[0].as<int32_t>(), ctx->gid[2].as<int32_t>(), flags.as<uint8_t>(),
                                ctx->stream));
        std::vector<uint8_t> hf((size_t)n4);
        HIPCHK(hipMemcpyAsync(hf.data(), flags.p, (size_t)n4, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        flags.release();
        std::vector<int32_t> run_of((size_t)n4), first;
        int32_t r = -1;
        for (int64_t q = 0; q < n4; ++q) {
            if (hf[q]) {
                ++r;
                first.push_back((int32_t)q);
            }
            run_of[q] = r;
        }
        const int64_t R = (int64_t)first.size();
        DevBuf dfirst;
        ALLOC(ctx->run_of4, sizeof(int32_t) * (size_t)n4);
        ALLOC(ctx->rtab, sizeof(float4) * (size_t)R);
        ALLOC(ctx->rz, sizeof(float) * (size_t)R);
        ALLOC(dfirst, sizeof(int32_t) * (size_t)R);
        HIPCHK(hipMemcpy(ctx->run_of4.p, run_of.data(), sizeof(int32_t) * (size_t)n4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(dfirst.p, first.data(), sizeof(int32_t) * (size_t)R, hipMemcpyHostToDevice));
        HIPCHK(launch_run_table(R, dfirst.as<int32_t>(), ctx->xi.as<float>(), ctx->zi.as<float>(), ctx->t1i.as<float>(),
                                ctx->t2i.as<float>(), ctx->dfi.as<float>(), ctx->rtab.as<float4>(), ctx->rz.as<float>(),
                                ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        ctx->n_runs = R;
    } else {
        ctx->run_of4.release();
        ctx->rtab.release();
        ctx->rz.release();
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    cleanup();
    ctx->axes = axes;
    ctx->Kint = kint;
    ctx->Kpad = Kpad;
    ctx->groups_valid = true;
    if (!ctx->has_seq) return GBS_OK;
    if (int rc = build_coil_layout(ctx)) return rc;
    return build_grouped_plan(ctx);
}

int gbs_get_info(gbs_ctx *ctx, gbs_info *info) {
    if (!ctx || !info) return GBS_E_INVALID;
    std::memset(info, 0, sizeof(*info));
    info->K = ctx->has_ph ? ctx->K : 0;
    info->n_blocks = ctx->has_seq ? (int64_t)ctx->seq.blocks.size() : 0;
    info->total_steps = ctx->has_seq ? ctx->seq.total_steps : 0;
    info->total_samples = ctx->has_seq ? ctx->seq.total_samples : 0;
    info->stepped_steps = ctx->has_seq ? ctx->seq.stepped_steps : 0;
    for (int a = 0; a < 3; ++a) info->n_groups[a] = ctx->groups_valid ? ctx->ng[a] : -1;
    info->groups_valid = ctx->groups_valid ? 1 : 0;
    info->device = ctx->device;
    info->n_tissue_groups = ctx->groups_valid ? ctx->n_tissue : -1;
    info->n_coils = ctx->n_coils;
    info->n_xz_groups = ctx->groups_valid ? ctx->n_runs : -1;
    return GBS_OK;
}

int gbs_plan_summary(const gbs_block *blocks, int64_t n_blocks, const float *rf_re, const float *rf_im,
                     const float *gx, const float *gy, const float *gz, int64_t total_steps,
                     const int32_t *adc_idx, int64_t total_samples, double dt, uint32_t axes, int64_t out[8]) {
    if (!out) return GBS_E_INVALID;
    std::string err;
    int rc = validate_sequence(blocks, n_blocks, total_steps, adc_idx, total_samples, dt, err);
    if (rc != GBS_OK) return rc;
    if (total_steps > 0 && (!rf_re || !rf_im || !gx || !gy || !gz)) return GBS_E_INVALID;
    HostSeq s;
    copy_sequence(s, blocks, n_blocks, rf_re, rf_im, gx, gy, gz, total_steps, adc_idx, total_samples, dt);
    Plan p = plan_grouped(s, classify(s), axes);
    out[0] = p.n_rf_grouped;
    out[1] = p.n_adc_grouped;
    out[2] = p.n_fallback;
    out[3] = p.n_b1zero;
    out[4] = p.n_passes + (p.final_pass ? 1 : 0);
    out[5] = p.n_emit_only;
    out[6] = (int64_t)p.rf.size();
    out[7] = p.n_relax;
    return GBS_OK;
}

int gbs_plan_cached_summary(const gbs_block *blocks, int64_t n_blocks, const float *rf_re, const float *rf_im,
                            const float *gx, const float *gy, const float *gz, int64_t total_steps,
                            const int32_t *adc_idx, int64_t total_samples, double dt, int64_t out[6]) {
    if (!out) return GBS_E_INVALID;
    std::string err;
    int rc = validate_sequence(blocks, n_blocks, total_steps, adc_idx, total_samples, dt, err);
    if (rc != GBS_OK) return rc;
    if (total_steps > 0 && (!rf_re || !rf_im || !gx || !gy || !gz)) return GBS_E_INVALID;
    HostSeq s;
    copy_sequence(s, blocks, n_blocks, rf_re, rf_im, gx, gy, gz, total_steps, adc_idx, total_samples, dt);
    Plan p = plan_cached(s, classify(s));
    int64_t adc_launches = 0;
    for (const Op &op : p.ops)
        if (op.kind == 3) ++adc_launches;
    out[0] = p.n_rf_cached;
    out[1] = (int64_t)p.rf.size();
    out[2] = p.n_adc_direct;
    out[3] = adc_launches;
    out[4] = p.n_fallback;
    out[5] = p.n_b1zero;
    return GBS_OK;
}

}  // extern "C"

// ----------------------------------------------------------------- simulate
namespace {

PlainArgs step_args(gbs_ctx *ctx, const StepOp &op, const PhantomPtrs &ph, int64_t K, const float *in_x,
                    const float *in_y, const float *in_z, float *ox, float *oy, float *oz) {
    PlainArgs a{};
    a.K = K;
    a.ph = ph;
    a.min_x = in_x;
    a.min_y = in_y;
    a.min_z = in_z;
    a.mout_x = ox;
    a.mout_y = oy;
    a.mout_z = oz;
    a.dt = ctx->seq.dt;
    a.gdt = kTwoPi * kGammaBar * ctx->seq.dt;
    a.has_pre = op.has_pre ? 1 : 0;
    a.pre_tau = op.pre.tau;
    for (int i = 0; i < 3; ++i) a.pre_cyc[i] = kGammaBar * op.pre.m[i];
    if (op.block >= 0) {
        const gbs_block &b = ctx->seq.blocks[op.block];
        a.wave = ctx->d_wave.as<StepW>() + b.step_offset + op.step_lo;
        a.n_steps = (int32_t)(op.step_hi - op.step_lo);
        a.sidx = ctx->d_adc.as<int32_t>() + b.sample_offset + op.sample_lo;
        a.step_base = (int32_t)op.step_lo;
        a.n_samples = op.sample_hi - op.sample_lo;
    } else {
        a.wave = ctx->d_wave.as<StepW>();
        a.n_steps = 0;
        a.sidx = ctx->d_adc.as<int32_t>();
        a.step_base = 0;
        a.n_samples = 0;
    }
    a.partial = ctx->partial;
    return a;
}

}  // namespace

// Samples per stepping launch: the coil sums share the launch's LDS accumulators.
static int32_t step_samples(const gbs_ctx *ctx) {
    return kMaxSamplesPerLaunch / (ctx->coil_re ? ctx->n_coils : 1);
}

// One stepping launch with its samples: the coil sums when the context has coil
// maps (sensitivities of the launch's isochromats: re + p * stride), then one
// finalize per coil into row p of the signal.
static int launch_steps(gbs_ctx *ctx, const PlainArgs &a, bool b1, int grid, const float *cre,
                        const float *cim, int64_t cstride, double *sig_out, int64_t first_sample) {
    const int32_t P = ctx->coil_re ? ctx->n_coils : 1;
    if (ctx->coil_re && a.n_samples > 0)
        HIPCHK(launch_plain_coils(a, PlainCoils{cre, cim, cstride, P}, b1, grid, ctx->stream));
    else
        HIPCHK(launch_plain(a, b1, grid, ctx->stream));
    for (int32_t p = 0; p < P && a.n_samples > 0; ++p)
        HIPCHK(launch_plain_finalize(ctx->partial + (size_t)p * grid * a.n_samples, grid, a.n_samples,
                                     sig_out + 2 * ((int64_t)p * ctx->seq.total_samples + first_sample), ctx->stream));
    return GBS_OK;
}

// Plain schedule (host only).
static void build_plain_plan(gbs_ctx *ctx) {
    ctx->pplan = plan_plain(ctx->seq, step_samples(ctx));
    if (ctx->pplan.ops.empty()) {  // still write (0, 0, M0) or the initial state out
        Op op;
        op.kind = 1;
        op.step = StepOp{};
        ctx->pplan.ops.push_back(op);
    }
    ctx->pplan_valid = true;
}

// Workspace of GBS_PLAIN: per-workgroup sample sums, and the FP64 state
// between launches when there is more than one.
static size_t plain_ws(const gbs_ctx *ctx, size_t *o_partial, size_t *o_state) {
    WsCarve w;
    *o_partial = w.take(sizeof(double2) * (size_t)plain_grid(ctx->K) * kMaxSamplesPerLaunch);
    *o_state = ctx->pplan.ops.size() > 1 ? w.take(sizeof(double) * 3 * (size_t)ctx->K) : 0;
    return w.off;
}

static int run_plain(gbs_ctx *ctx, char *ws, const float *m_init, float *m_out, double *sig_out, gbs_stats *st) {
    const int64_t K = ctx->K;
    const Plan &plan = ctx->pplan;
    const int grid = plain_grid(K);
    size_t o_partial = 0, o_state = 0;
    plain_ws(ctx, &o_partial, &o_state);
    ctx->partial = (double2 *)(ws + o_partial);
    float *ox = m_out, *oy = m_out + K, *oz = m_out + 2 * K;
    // the state stays in FP64 between launches and is rounded to the FP32
    // output once, in the last launch
    double *sx = nullptr, *sy = nullptr, *sz = nullptr;
    if (plan.ops.size() > 1) {
        sx = (double *)(ws + o_state);
        sy = sx + K;
        sz = sx + 2 * K;
    }
    bool first = true;
    for (size_t oi = 0; oi < plan.ops.size(); ++oi) {
        const Op &op = plan.ops[oi];
        const bool last = oi + 1 == plan.ops.size();
        const float *ix = first && m_init ? m_init : (first ? nullptr : ox);
        const float *iy = first && m_init ? m_init + K : (first ? nullptr : oy);
        const float *iz = first && m_init ? m_init + 2 * K : (first ? nullptr : oz);
        PlainArgs a = step_args(ctx, op.step, ctx->ph, K, ix, iy, iz, ox, oy, oz);
        if (sx) {
            if (!first) {
                a.min_x = a.min_y = a.min_z = nullptr;
                a.min64_x = sx;
                a.min64_y = sy;
                a.min64_z = sz;
            }
            if (!last) {
                a.mout_x = a.mout_y = a.mout_z = nullptr;
                a.mout64_x = sx;
                a.mout64_y = sy;
                a.mout64_z = sz;
            }
        }
        const bool b1 = op.step.block >= 0 && ctx->cls[op.step.block].has_b1;
        const int64_t s0 = op.step.block >= 0 ? ctx->seq.blocks[op.step.block].sample_offset + op.step.sample_lo : 0;
        if (int rc = launch_steps(ctx, a, b1, grid, ctx->coil_re, ctx->coil_im, K, sig_out, s0)) return rc;
        first = false;
    }
    if (st) st->n_fallback = 0;
    return GBS_OK;
}

// Build the cached grouped plan: schedule, arena layout, sample tables and
// job arrays (device).  Host work only once per (sequence, groups).
// Do raster steps [step_offset, step_offset + n_steps) play exactly the
// surrogate's pulse (Gz-only, bit for bit)?
static bool matches_pulse(const gbs_ctx *ctx, int64_t step_offset, int64_t n_steps) {
    const gbs_mlp *m = ctx->mlp;
    const HostSeq &s = ctx->seq;
    if (!m || !m->has_pulse || m->device != ctx->device || n_steps != m->n_steps || s.dt != m->dt) return false;
    const size_t o = (size_t)step_offset, n = (size_t)n_steps;
    for (size_t i = 0; i < n; ++i)
        if (s.gx[o + i] != 0.f || s.gy[o + i] != 0.f) return false;
    return std::memcmp(&s.rf_re[o], m->rf_re.data(), n * sizeof(float)) == 0 &&
           std::memcmp(&s.rf_im[o], m->rf_im.data(), n * sizeof(float)) == 0 &&
           std::memcmp(&s.gz[o], m->gz.data(), n * sizeof(float)) == 0;
}

// Algorithmic HBM bytes per isochromat of one sweep launch: the state it
// reads (none when it starts from (0, 0, M0)), M0 and the per-isochromat
// arrays its ops need, and the state it writes (a 16-byte row in the last
// launch of a run).
static double sweep_bytes_per_iso(int need, bool write_m, bool fresh, bool final_rows) {
    double b = fresh ? 0.0 : 8.0;
    if (need & kNeedMz) b += fresh ? 4.0 : 8.0;
    if (need & kNeedRun) b += 1.0;  // one int32 per 4 isochromats
    b += 4.0 * (!!(need & kNeedGx) + !!(need & kNeedGy) + !!(need & kNeedGz) + !!(need & kNeedY) + !!(need & kNeedZ));
    if (write_m) b += final_rows ? 16.0 : ((need & kNeedMz) ? 12.0 : 8.0);
    return b;
}

// Does a sweep with these needs run in the emission-only kernel (launch_sweep)?
static bool in_emit_kernel(int need, bool coils) {
    return (need & kEmitOnly) && !coils && !(need & (kNeedGy | kNeedZ | kForceGeneral));
}

// Does a sweep with these needs run in a kernel of 8 isochromats per thread
// that can write per-wavefront partial sums (k_sweep, k_sweep_pairs,
// k_sweep_emit), i.e. not the general or the coil sweep?
static bool in_partial_kernel(int need, bool coils) {
    return !coils && !(need & (kNeedGy | kNeedZ | kForceGeneral));
}

static int build_grouped_plan(gbs_ctx *ctx) {
    GroupedPlan &g = ctx->gp;
    const HostSeq &s = ctx->seq;
    g = GroupedPlan{};
    g.plan = plan_grouped(s, ctx->cls, ctx->axes, step_samples(ctx));
    const Plan &plan = g.plan;
    g.zbuilt = (ctx->axes & GBS_AX_Z) != 0;
    if (ctx->mlp && ctx->mlp->device == ctx->device) {
        for (size_t i = 0; i < plan.rf.size(); ++i)
            if (plan.rf[i].axis == 2 && matches_pulse(ctx, plan.rf[i].step_offset, plan.rf[i].n_steps)) {
                g.surr_rf = (int)i;
                break;
            }
    }
    const int64_t Gx = ctx->ng[0], Gz = g.zbuilt ? ctx->ng[2] : 0;

    // ---- arena: FP64 combined transitions, folded transitions, map tables
    size_t off = 0;
    g.rf_off.resize(plan.rf.size());
    g.expand.clear();
    g.pair_jobs.clear();
    // groups behind the transition rows of an op's rf_axis (kPairRows: two-axis groups)
    auto rows_groups = [&](int A) { return A == kPairRows ? ctx->n_runs : ctx->ng[A]; };
    auto rows_table = [&](int A) { return A == kPairRows ? ctx->rtab.as<float4>() : ctx->gtab[A].as<float4>(); };
    std::vector<size_t> comp_off(plan.rf.size());
    for (size_t i = 0; i < plan.rf.size(); ++i) {
        const bool tissue = plan.rf[i].axis == kTissueAxis;
        const int64_t G = tissue ? ctx->n_tissue : plan.rf[i].axis == kPairAxis ? ctx->n_runs : ctx->ng[plan.rf[i].axis];
        comp_off[i] = off;
        if (plan.rf[i].axis != kPairAxis) g.max_rf_groups = std::max(g.max_rf_groups, G);  // k_compose's grid
        off = align256(off + sizeof(double) * 12 * (size_t)G);
        g.rf_off[i] = comp_off[i];
        if (plan.rf[i].axis == kPairAxis) g.pair_jobs.emplace_back(comp_off[i], (int)i);
        if (tissue) {  // expanded to x-group rows for the fold
            g.rf_off[i] = off;
            off = align256(off + sizeof(double) * 12 * (size_t)Gx);
            g.expand.emplace_back(comp_off[i], g.rf_off[i]);
        }
    }
    // Map-factor tables.  Ops whose factors have the same kind, duration and
    // moment (the echoes and shots of a repeated timing) share one table:
    // equal inputs give equal entries.  (`out` holds the arena offset until
    // the offsets are made workspace-relative below.)
    std::vector<TabJob> tjobs;
    auto table = [&](int kind, int64_t n, double tau, double cyc, size_t row_bytes) {
        for (const TabJob &t : tjobs)
            if (t.kind == kind && t.n == (int32_t)n && t.tau == tau && t.cyc == cyc) return (size_t)t.out;
        const size_t o = off;
        off = align256(off + row_bytes * (size_t)n);
        tjobs.push_back(TabJob{kind, (int32_t)n, tau, cyc, (void *)o});
        return o;
    };
    auto x_table = [&](int kind, double tau, double cyc) { return table(kind, Gx, tau, cyc, sizeof(float4)); };
    auto z_table = [&](double cyc) { return table(1, Gz, 0.0, cyc, sizeof(float2)); };
    struct FoldPlan {
        size_t out_off;
        int axis, rf_id, has_pre;
        double tau, cyc;
    };
    std::vector<FoldPlan> folds;
    const size_t kNone = ~(size_t)0;
    struct OpTabs {  // arena offsets of one op's tables
        size_t pre_x = kNone, pre_z = kNone, ttab = kNone, emit_x = kNone, emit_z = kNone;
    };
    std::vector<PassOp> passes;  // grouped ops in schedule order, final map last
    std::vector<int> pass_of_op(plan.ops.size(), -1);
    for (size_t i = 0; i < plan.ops.size(); ++i)
        if (plan.ops[i].kind == 0) {
            pass_of_op[i] = (int)passes.size();
            passes.push_back(plan.ops[i].pass);
        }
    if (plan.final_pass) {
        PassOp f;
        f.has_pre = true;
        f.pre = plan.final_map;
        f.write_m = true;
        passes.push_back(f);
    }
    std::vector<OpTabs> ot(passes.size());
    for (size_t i = 0; i < passes.size(); ++i) {
        const PassOp &p = passes[i];
        if (p.rf_axis >= 0) {
            // the tissue part and the own-axis phase of the pre map fold into T'
            const int A = p.rf_axis;
            // (two-axis groups fold the x phase; their z phase stays a z-group table).
            // Ops with the same transition and the same folded part share one table.
            const double cyc = kGammaBar * p.pre.m[A == kPairRows ? 0 : A];
            const int hp = p.has_pre ? 1 : 0;
            const double tau = p.has_pre ? p.pre.tau : 0.0, fc = p.has_pre ? cyc : 0.0;
            auto same = [&](const FoldPlan &f) {
                return f.axis == A && f.rf_id == p.rf_id && f.has_pre == hp && f.tau == tau && f.cyc == fc;
            };
            const auto hit = std::find_if(folds.begin(), folds.end(), same);
            if (hit != folds.end()) {
                ot[i].ttab = hit->out_off;
            } else {
                ot[i].ttab = off;
                off = align256(off + sizeof(float4) * 3 * (size_t)rows_groups(A));
                folds.push_back(FoldPlan{ot[i].ttab, A, p.rf_id, hp, tau, fc});
            }
            if (p.has_pre) {
                if (A != 0 && A != kPairRows && p.pre.m[0] != 0.0) ot[i].pre_x = x_table(2, 0.0, kGammaBar * p.pre.m[0]);
                if (A != 2 && g.zbuilt && p.pre.m[2] != 0.0) ot[i].pre_z = z_table(kGammaBar * p.pre.m[2]);
            }
        } else if (p.has_pre) {
            ot[i].pre_x = x_table(0, p.pre.tau, kGammaBar * p.pre.m[0]);
            if (g.zbuilt && p.pre.m[2] != 0.0) ot[i].pre_z = z_table(kGammaBar * p.pre.m[2]);
        }
        if (p.emit_axis >= 0) {
            ot[i].emit_x = x_table(0, p.emit.tau, kGammaBar * p.emit.m[0]);
            if (g.zbuilt && p.emit.m[2] != 0.0) ot[i].emit_z = z_table(kGammaBar * p.emit.m[2]);
        }
    }
    const size_t tab_bytes = off;
    g.max_tab = std::max<int64_t>(Gx, Gz);

    size_t goff = 0, soff = 0;
    g.gsum_off.resize(plan.adc.size());
    std::vector<size_t> samp_off(plan.adc.size());
    for (size_t i = 0; i < plan.adc.size(); ++i) {
        const AdcJob &j = plan.adc[i];
        g.gsum_off[i] = goff;
        goff += (size_t)ctx->ng[j.axis] * (size_t)ctx->n_coils;  // one block of sums per coil
        samp_off[i] = soff;
        soff += (size_t)s.blocks[j.block].n_samples;
        g.max_adc_groups = std::max(g.max_adc_groups, (int)ctx->ng[j.axis]);
        g.max_adc_samples = std::max(g.max_adc_samples, (int)s.blocks[j.block].n_samples);
    }
    g.gsum_count = goff;
    WsCarve w;
    g.w_state = w.take(28 * (size_t)ctx->Kpad);  // mx, my, mz planes (4 B each), final rows (16 B)
    g.w_tabs = w.take(tab_bytes);
    g.w_gsum = w.take(sizeof(double2) * goff);
    if (plan.n_fallback) g.w_partial = w.take(sizeof(double2) * (size_t)plain_grid(ctx->Kint) * kMaxSamplesPerLaunch);
    ALLOC(ctx->samp, sizeof(double2) * std::max<size_t>(soff, 1));
    // workspace-relative addresses in the table arena and the group sums
    auto tb = [&](size_t o) { return ws_rel<char>(g.w_tabs + o); };
    auto gsum_at = [&](size_t i) { return ws_rel<double2>(g.w_gsum + sizeof(double2) * i); };
    for (auto &t : tjobs) t.out = tb((size_t)t.out);

    // per-sample tables (tau_n, gamma_bar m_n) of the grouped with-ADC blocks (Eq. 10)
    std::vector<double2> &hs = ctx->host_samp;
    hs.assign(soff, double2{0.0, 0.0});
    for (size_t i = 0; i < plan.adc.size(); ++i) {
        const AdcJob &j = plan.adc[i];
        const gbs_block &b = s.blocks[j.block];
        const std::vector<float> &gw = j.axis == 0 ? s.gx : j.axis == 1 ? s.gy : s.gz;
        double m = 0.0;
        int64_t step = 0;
        for (int32_t n = 0; n < b.n_samples; ++n) {
            const int32_t tgt = s.adc_idx[b.sample_offset + n];
            for (; step < tgt; ++step) m += (double)gw[b.step_offset + step] * s.dt;
            hs[samp_off[i] + n] = double2{(double)tgt * s.dt, kGammaBar * m};
        }
    }

    // ---- job arrays
    std::vector<RfJobDev> rj(plan.rf.size());
    for (size_t i = 0; i < plan.rf.size(); ++i) {
        const RfJob &r = plan.rf[i];
        // the surrogate's transition is not composed here (n_groups = 0 skips it)
        if (r.axis == kPairAxis) {  // composed by its own kernel (k_compose_pair)
            rj[i] = RfJobDev{0, (int32_t)r.n_steps, 0, ctx->d_wave.as<StepW>() + r.step_offset, nullptr,
                             (double *)tb(comp_off[i])};
            continue;
        }
        if (r.axis == kTissueAxis) {  // no gradients: the coordinate column of the table is unused
            rj[i] = RfJobDev{0, (int32_t)r.n_steps, ctx->n_tissue, ctx->d_wave.as<StepW>() + r.step_offset,
                             ctx->ttab.as<float4>(), (double *)tb(comp_off[i])};
            continue;
        }
        rj[i] = RfJobDev{r.axis, (int32_t)r.n_steps, ctx->ng[r.axis], ctx->d_wave.as<StepW>() + r.step_offset,
                         ctx->gtab[r.axis].as<float4>(), (double *)tb(g.rf_off[i])};
    }
    std::vector<RfJobDev> rj_surr(rj);  // GBS_SURROGATE: the network's transition is not composed
    if (g.surr_rf >= 0) rj_surr[g.surr_rf].n_groups = 0;
    if (g.surr_rf >= 0) {
        // tuples, network output, spot-check indices (seeded, distinct) and exact values
        const int64_t G = ctx->ng[2];
        g.surr_groups = G;
        g.surr_n_check = (int)std::min<int64_t>(ctx->surr_check, G);
        size_t so = 0;
        auto take = [&](size_t bytes) {
            const size_t o = so;
            so = align256(so + bytes);
            return o;
        };
        g.s_tuples = take(sizeof(float) * 5 * (size_t)G);
        g.s_T32 = take(sizeof(float) * 12 * (size_t)G);
        g.s_exact = take(sizeof(double) * 12 * (size_t)g.surr_n_check);
        g.s_res = take(sizeof(float));
        g.s_fb = take(sizeof(int32_t));
        std::vector<int32_t> all((size_t)G);
        for (int64_t i = 0; i < G; ++i) all[i] = (int32_t)i;
        uint64_t rs = ctx->surr_seed ^ 0x5DEECE66Dull;
        for (int k = 0; k < g.surr_n_check; ++k) {  // partial Fisher-Yates
            rs = rs * 6364136223846793005ull + 1442695040888963407ull;
            const int64_t j = k + (int64_t)((rs >> 33) % (uint64_t)(G - k));
            std::swap(all[k], all[j]);
        }
        g.w_surr = w.take(so);
        ALLOC(ctx->surr_idx, sizeof(int32_t) * (size_t)g.surr_n_check);
        HIPCHK(hipMemcpy(ctx->surr_idx.p, all.data(), sizeof(int32_t) * g.surr_n_check, hipMemcpyHostToDevice));
    }
    std::vector<FoldJob> fj(folds.size());
    for (size_t i = 0; i < folds.size(); ++i) {
        const FoldPlan &f = folds[i];
        fj[i] = FoldJob{f.axis, f.has_pre, rows_groups(f.axis), (const double *)tb(g.rf_off[f.rf_id]),
                        rows_table(f.axis), f.tau, f.cyc, (float4 *)tb(f.out_off)};
        g.max_fold_groups = std::max(g.max_fold_groups, rows_groups(f.axis));
    }
    // readouts whose sample times and moments are arithmetic in the sample index take the
    // geometric-sequence evaluation; the rest the direct one
    std::vector<AdcJobDev> aj;
    std::vector<AdcLinJob> lj;
    g.max_adc_groups = 0;
    g.max_adc_samples = 0;
    for (size_t i = 0; i < plan.adc.size(); ++i) {
        const AdcJob &j = plan.adc[i];
        const gbs_block &b = s.blocks[j.block];
        const int ns = b.n_samples;
        const double2 *h = hs.data() + samp_off[i];
        bool lin = ns >= 1;
        double dtau = 0.0, dcyc = 0.0;
        if (ns >= 2) {
            dtau = (h[ns - 1].x - h[0].x) / (ns - 1);
            dcyc = (h[ns - 1].y - h[0].y) / (ns - 1);
            for (int n = 0; n < ns && lin; ++n) {
                // phase error of the linear model below 1e-9 cycles per metre and 1e-15 s
                lin = std::fabs(h[n].x - (h[0].x + n * dtau)) <= 1e-15 &&
                      std::fabs(h[n].y - (h[0].y + n * dcyc)) <= 1e-9;
            }
        }
        // coil p: its own block of group sums, its own row of the signal
        for (int32_t p = 0; p < ctx->n_coils; ++p) {
            const double2 *gs = gsum_at(g.gsum_off[i] + (size_t)p * (size_t)ctx->ng[j.axis]);
            const int64_t so = (int64_t)p * s.total_samples + b.sample_offset;
            if (lin) {
                lj.push_back(AdcLinJob{ns, (int32_t)ctx->ng[j.axis], gs, ctx->gtab[j.axis].as<float4>(), h[0].x,
                                       dtau, h[0].y, dcyc, so});
                g.max_adclin_groups = std::max(g.max_adclin_groups, (int)ctx->ng[j.axis]);
            } else {
                aj.push_back(AdcJobDev{ns, (int32_t)ctx->ng[j.axis], gs, ctx->gtab[j.axis].as<float4>(),
                                       ctx->samp.as<double2>() + samp_off[i], so});
                g.max_adc_groups = std::max(g.max_adc_groups, (int)ctx->ng[j.axis]);
                g.max_adc_samples = std::max(g.max_adc_samples, ns);
            }
        }
    }

    // ---- sweep ops: grouped ops in schedule order; consecutive ones fuse
    auto ptr4 = [&](size_t o) { return o == kNone ? (const float4 *)nullptr : (const float4 *)tb(o); };
    auto ptr2 = [&](size_t o) { return o == kNone ? (const float2 *)nullptr : (const float2 *)tb(o); };
    std::vector<SweepOp> sops;
    std::vector<int> op_need;       // per sweep op: arrays it needs
    std::vector<double> op_flops;   // per sweep op: algorithmic flops per isochromat
    auto add_op = [&](int pi) {
        const PassOp &p = passes[pi];
        const OpTabs &t = ot[pi];
        SweepOp o{};
        o.rf_axis = p.rf_axis;
        o.emit_axis = p.emit_axis;
        double fl = 0.0;
        if (p.has_pre) {
            const int A = p.rf_axis;  // -1: nothing folded
            o.pre_xtab = ptr4(t.pre_x);
            o.pre_ztab = ptr2(t.pre_z);
            o.pre_cy = (A != 1) ? kGammaBar * p.pre.m[1] : 0.0;
            o.pre_cz = (A != 2 && !g.zbuilt) ? kGammaBar * p.pre.m[2] : 0.0;
            const int nf = (o.pre_xtab != nullptr) + (o.pre_ztab != nullptr) + (o.pre_cy != 0.0) + (o.pre_cz != 0.0);
            if (nf) {
                o.flags |= kOpPre;
                fl += 6.0 * nf;
            }
            if (A < 0) {
                o.flags |= kPreMz;
                fl += 3.0;
            }
        }
        if (p.rf_axis >= 0) {
            o.flags |= kOpRf;
            o.ttab = ptr4(t.ttab);
            fl += 24.0;
        }
        if (p.emit_axis >= 0) {
            o.flags |= kOpEmit;
            o.emit_xtab = ptr4(t.emit_x);
            o.emit_ztab = ptr2(t.emit_z);
            o.emit_cy = kGammaBar * p.emit.m[1];
            o.emit_cz = g.zbuilt ? 0.0 : kGammaBar * p.emit.m[2];
            o.gsum = gsum_at(g.gsum_off[p.adc_job]);
            o.gsum_stride = (int32_t)ctx->ng[p.emit_axis];
            fl += 8.0 + 6.0 * ((o.emit_ztab != nullptr) + (o.emit_cy != 0.0) + (o.emit_cz != 0.0));
        }
        int need = 0;
        if ((o.flags & kOpRf) || (o.flags & kPreMz)) need |= kNeedMz;
        if (o.pre_xtab || (o.flags & kOpEmit) || p.rf_axis == 0) need |= kNeedGx;
        if (p.rf_axis == 1 || p.emit_axis == 1) need |= kNeedGy;
        if (p.rf_axis == kPairRows) need |= kNeedRun;
        if (o.pre_ztab || o.emit_ztab || p.rf_axis == 2 || p.emit_axis == 2) need |= kNeedGz;
        if (o.pre_cy != 0.0 || o.emit_cy != 0.0) need |= kNeedY;
        if (o.pre_cz != 0.0 || o.emit_cz != 0.0) need |= kNeedZ;
        if (g.segs.empty() || g.exec.empty() || g.exec.back().first != 0) {
            g.segs.push_back(GroupedPlan::Seg{(int)sops.size(), (int)sops.size(), 0, false, 0.0, 0.0});
            g.exec.push_back({0, (int)g.segs.size() - 1});
        }
        GroupedPlan::Seg &sg = g.segs.back();
        sg.op_end = (int)sops.size() + 1;
        sg.need |= need;
        sg.write_m = sg.write_m || (o.flags & (kOpPre | kOpRf));
        sg.flops_per_iso += fl;
        sops.push_back(o);
        op_need.push_back(need);
        op_flops.push_back(fl);
    };
    for (size_t i = 0; i < plan.ops.size(); ++i) {
        if (plan.ops[i].kind == 0)
            add_op(pass_of_op[i]);
        else
            g.exec.push_back({1, (int)i});
    }
    if (plan.final_pass) add_op((int)passes.size() - 1);

    // Runs of at least kEmitRun emissions that leave the state alone (an EPI
    // readout train) become sweeps of their own: the state is written once
    // before them, and they run in the emission-only kernel, whose few live
    // registers allow more waves per SIMD to hide the per-op load latency.
    {
        constexpr int kEmitRun = 16;
        auto emit_only = [&](int o) {
            return (sops[o].flags & kOpEmit) && !(sops[o].flags & (kOpPre | kOpRf | kPreMz));
        };
        std::vector<GroupedPlan::Seg> segs;
        std::vector<int> remap(g.segs.size() + 1, 0);
        std::vector<std::vector<int>> pieces(g.segs.size());
        for (size_t si = 0; si < g.segs.size(); ++si) {
            const GroupedPlan::Seg &sg = g.segs[si];
            int o = sg.op_begin;
            while (o < sg.op_end) {
                int e = o;
                while (e < sg.op_end && emit_only(e)) ++e;
                const bool run = e - o >= kEmitRun;
                if (!run) {  // up to the next long emission run
                    e = o + 1;
                    while (e < sg.op_end) {
                        int f = e;
                        while (f < sg.op_end && emit_only(f)) ++f;
                        if (f - e >= kEmitRun) break;
                        e = f > e ? f : e + 1;
                    }
                }
                GroupedPlan::Seg piece{o, e, 0, false, 0.0, 0.0};
                for (int q = o; q < e; ++q) {
                    piece.need |= op_need[q];
                    piece.write_m = piece.write_m || (sops[q].flags & (kOpPre | kOpRf));
                    piece.flops_per_iso += op_flops[q];
                }
                if (run) piece.need |= kEmitOnly;
                // a lone closed-form map that ends the segment (the final
                // relaxation) rides along with the emission run before it
                const int t = e;
                if (run && t + 1 == sg.op_end && (sops[t].flags & kOpPre) && !(sops[t].flags & (kOpRf | kOpEmit)) &&
                    !(op_need[t] & (kNeedGy | kNeedZ | kNeedRun))) {
                    piece.op_end = t + 1;
                    piece.need |= op_need[t] | kEmitTail;
                    piece.write_m = true;
                    piece.flops_per_iso += op_flops[t];
                    e = t + 1;
                }
                pieces[si].push_back((int)segs.size());
                segs.push_back(piece);
                o = e;
            }
            // a few general ops right before an emission run (the excitation and
            // the first readout's pre map) join it as its head (kEmitHead), so the
            // state is not written and read once more between them
            auto head_ok = [&](int q) {
                const SweepOp &op = sops[q];
                if (op_need[q] & (kNeedGy | kNeedZ | kNeedRun)) return false;
                if ((op.flags & kOpRf) && op.rf_axis != 0 && op.rf_axis != 2) return false;
                if ((op.flags & kOpEmit) && op.emit_axis != 0 && op.emit_axis != 2) return false;
                return true;
            };
            std::vector<int> &pl = pieces[si];
            for (size_t k = 0; k + 1 < pl.size(); ++k) {
                GroupedPlan::Seg &h = segs[pl[k]], &r = segs[pl[k + 1]];
                if ((h.need & kEmitOnly) || !(r.need & kEmitOnly) || (r.need & kEmitHead)) continue;
                const int n = h.op_end - h.op_begin;
                int n_em = 0;
                bool ok = n <= 4;
                for (int q = h.op_begin; ok && q < h.op_end; ++q) {
                    ok = head_ok(q);
                    n_em += (sops[q].flags & kOpEmit) ? 1 : 0;
                }
                if (!ok || n_em > 1) continue;
                r.op_begin = h.op_begin;
                r.n_head = n;
                r.need |= h.need | kEmitHead;
                r.write_m = r.write_m || h.write_m;
                r.flops_per_iso += h.flops_per_iso;
                pl.erase(pl.begin() + (long)k);
            }
        }
        // keep only the pieces still in use (a merged head's own piece is not)
        std::vector<GroupedPlan::Seg> used;
        std::vector<int> renum(segs.size(), -1);
        for (auto &pl : pieces)
            for (int &pi : pl) {
                if (renum[pi] < 0) {
                    renum[pi] = (int)used.size();
                    used.push_back(segs[pi]);
                }
                pi = renum[pi];
            }
        std::vector<std::pair<int, int>> exec;
        for (const auto &it : g.exec) {
            if (it.first != 0) {
                exec.push_back(it);
                continue;
            }
            for (int pi : pieces[it.second]) exec.push_back({0, pi});
        }
        g.segs.swap(used);
        g.exec.swap(exec);
    }

    // y phases of consecutive emissions inside a sweep: direct evaluation, or
    // a complex recurrence when the coefficients step evenly (restarted every
    // 16 emissions to bound FP32 drift).  The kernel keeps the step factor
    // between chains, so a chain with the step of the last one reuses it.
    // (The head ops of an emission sweep keep their own chains: the emission
    // kernel starts its recurrence after them.)
    std::vector<std::pair<int, int>> ranges;
    for (const auto &sg : g.segs) {
        if (sg.n_head) {
            ranges.push_back({sg.op_begin, sg.op_begin + sg.n_head});
            ranges.push_back({sg.op_begin + sg.n_head, sg.op_end});
        } else {
            ranges.push_back({sg.op_begin, sg.op_end});
        }
    }
    for (const auto &rg : ranges) {
        double prev = 0.0, step = 0.0, held = 0.0;  // held: step the kernel's factor holds (starts at 1)
        bool have_prev = false, have_step = false;
        int chain = 0;
        std::vector<int> em;
        for (int o = rg.first; o < rg.second; ++o)
            if (sops[o].flags & kOpEmit) em.push_back(o);
        for (size_t e = 0; e < em.size(); ++e) {
            SweepOp &o = sops[em[e]];
            const double c = o.emit_cy;
            if (c == 0.0) {
                have_prev = have_step = false;
                continue;
            }
            const bool stepped = have_prev && have_step && chain < 15 &&
                                 std::fabs(c - prev - step) <= 1e-12 * std::max(std::fabs(step), std::fabs(c));
            if (stepped) {
                o.flags |= kYStep;
                ++chain;
            } else {
                o.flags |= kYDirect;
                chain = 0;
                have_step = false;
                if (e + 1 < em.size() && sops[em[e + 1]].emit_cy != 0.0) {
                    step = sops[em[e + 1]].emit_cy - c;
                    have_step = true;
                    if (std::fabs(step - held) > 1e-12 * std::fabs(step)) {
                        o.flags |= kYSetR;
                        o.emit_dcy = step;
                        held = step;
                    } else {
                        step = held;
                    }
                }
            }
            prev = c;
            have_prev = true;
        }
        // chain lengths for the emission-only sweep: stepped emissions after each direct one
        for (size_t e = 0; e < em.size(); ++e) {
            SweepOp &o = sops[em[e]];
            if (!(o.flags & kYDirect)) continue;
            int n = 0;
            while (e + 1 + n < em.size() && em[e + 1 + n] == em[e] + 1 + n && (sops[em[e + 1 + n]].flags & kYStep)) ++n;
            if (n > kChainMask) n = kChainMask;
            o.flags |= n << kChainShift;
        }
    }
    // a sweep whose emissions need no recurrence holds a repeated pre-map y
    // phase in the recurrence's factor instead of evaluating it per op.  A
    // stepped emission needs the factor even without kYSetR: a chain whose
    // step is zero (emissions at the same y moment) multiplies by the 1 the
    // factor starts with.
    for (const auto &sg : g.segs) {
        bool free_factor = true;
        for (int o = sg.op_begin; o < sg.op_end; ++o)
            free_factor = free_factor && !(sops[o].flags & (kYSetR | kYStep));
        if (!free_factor) continue;
        double held = 0.0;
        bool have = false;
        for (int o = sg.op_begin; o < sg.op_end; ++o) {
            SweepOp &op = sops[o];
            if (!(op.flags & kOpPre) || op.pre_cy == 0.0) continue;
            if (have && std::fabs(op.pre_cy - held) <= 1e-12 * std::fabs(op.pre_cy)) {
                op.flags |= kPreYHold;
            } else {
                op.flags |= kPreYSet;
                held = op.pre_cy;
                have = true;
            }
        }
    }
    // x-group sums of the emissions through per-wavefront partials
    // (kPartials) instead of memory-side atomics, one PartJob per emission,
    // in every segment that runs in a kernel of 8 isochromats per thread
    std::vector<PartJob> pj;
    {
        const int64_t n_waves = 4 * ((ctx->Kint / 8 + 255) / 256);  // 8 isochromats per thread
        int64_t n_part = 0;
        const bool coils = ctx->coil_re != nullptr;
        for (const auto &sg : g.segs)
            if (in_partial_kernel(sg.need, coils))
                for (int o = sg.op_begin; o < sg.op_end; ++o)
                    if ((sops[o].flags & kOpEmit) && sops[o].emit_axis == 0) ++n_part;
        if (n_part) g.w_part = w.take(sizeof(float4) * (size_t)n_waves * (size_t)n_part);
        int64_t k = 0;
        g.seg_parts.assign(g.segs.size(), {0, 0});
        for (size_t si = 0; si < g.segs.size(); ++si) {
            GroupedPlan::Seg &sg = g.segs[si];
            if (!in_partial_kernel(sg.need, coils)) continue;
            const int first = (int)pj.size();
            for (int o = sg.op_begin; o < sg.op_end; ++o) {
                SweepOp &op = sops[o];
                if (!(op.flags & kOpEmit) || op.emit_axis != 0) continue;
                op.part = ws_rel<float4>(g.w_part + sizeof(float4) * (size_t)n_waves * (size_t)k++);
                pj.push_back(PartJob{op.part, op.gsum});
            }
            if ((int)pj.size() > first) {
                sg.need |= kPartials;
                g.seg_parts[si] = {first, (int)pj.size() - first};
            }
        }
    }
    g.ws_bytes = w.off;
    for (auto &sg : g.segs) sg.bytes_per_iso = sweep_bytes_per_iso(sg.need, sg.write_m, false, false);
    g.n_ops = (int64_t)sops.size();

    g.n_rf = (int)rj.size();
    g.n_fold = (int)fj.size();
    g.n_tab = (int)tjobs.size();
    g.n_adc = (int)aj.size();
    g.n_adclin = (int)lj.size();
    g.o_rf = 0;
    g.o_rf_surr = align256(sizeof(RfJobDev) * rj.size());
    g.o_fold = g.o_rf_surr + align256(sizeof(RfJobDev) * rj.size());
    g.o_tab = g.o_fold + align256(sizeof(FoldJob) * fj.size());
    g.o_adc = g.o_tab + align256(sizeof(TabJob) * tjobs.size());
    g.o_adclin = g.o_adc + align256(sizeof(AdcJobDev) * aj.size());
    g.o_sweep = g.o_adclin + align256(sizeof(AdcLinJob) * lj.size());
    g.o_part = g.o_sweep + align256(sizeof(SweepOp) * sops.size());
    const size_t jbytes = g.o_part + sizeof(PartJob) * pj.size();
    ctx->host_jobs.assign(jbytes, 0);
    auto put = [&](size_t o, const void *src, size_t n) {
        if (n) std::memcpy(ctx->host_jobs.data() + o, src, n);
    };
    put(g.o_rf, rj.data(), sizeof(RfJobDev) * rj.size());
    put(g.o_rf_surr, rj_surr.data(), sizeof(RfJobDev) * rj_surr.size());
    put(g.o_fold, fj.data(), sizeof(FoldJob) * fj.size());
    put(g.o_tab, tjobs.data(), sizeof(TabJob) * tjobs.size());
    put(g.o_adc, aj.data(), sizeof(AdcJobDev) * aj.size());
    put(g.o_adclin, lj.data(), sizeof(AdcLinJob) * lj.size());
    put(g.o_sweep, sops.data(), sizeof(SweepOp) * sops.size());
    put(g.o_part, pj.data(), sizeof(PartJob) * pj.size());
    // the pointer fields that hold workspace offsets
    const std::vector<char> &img = ctx->host_jobs;
    add_relocs<RfJobDev>(g.relocs, img, g.o_rf, rj.size(), {offsetof(RfJobDev, out)});
    add_relocs<RfJobDev>(g.relocs, img, g.o_rf_surr, rj_surr.size(), {offsetof(RfJobDev, out)});
    add_relocs<FoldJob>(g.relocs, img, g.o_fold, fj.size(), {offsetof(FoldJob, t64), offsetof(FoldJob, out)});
    add_relocs<TabJob>(g.relocs, img, g.o_tab, tjobs.size(), {offsetof(TabJob, out)});
    add_relocs<AdcJobDev>(g.relocs, img, g.o_adc, aj.size(), {offsetof(AdcJobDev, gsum)});
    add_relocs<AdcLinJob>(g.relocs, img, g.o_adclin, lj.size(), {offsetof(AdcLinJob, gsum)});
    add_relocs<SweepOp>(g.relocs, img, g.o_sweep, sops.size(),
                        {offsetof(SweepOp, pre_xtab), offsetof(SweepOp, part), offsetof(SweepOp, pre_ztab),
                         offsetof(SweepOp, ttab), offsetof(SweepOp, emit_xtab), offsetof(SweepOp, emit_ztab),
                         offsetof(SweepOp, gsum)});
    add_relocs<PartJob>(g.relocs, img, g.o_part, pj.size(), {offsetof(PartJob, part), offsetof(PartJob, gsum)});
    ALLOC(ctx->jobs, jbytes);
    g.uploaded_ws = nullptr;
    if (soff) HIPCHK(hipMemcpy(ctx->samp.p, hs.data(), sizeof(double2) * soff, hipMemcpyHostToDevice));
    // GBS_PROFILE events: a (start, stop) pair per sweep
    while (ctx->pev.size() < 2 * (g.segs.size() + 1)) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        ctx->pev.push_back(e);
    }
    g.valid = true;
    return GBS_OK;
}

// Device copy of the grouped job descriptors with their workspace offsets
// turned into addresses in `ws`; done again only when the workspace moves.
static int relocate_jobs(gbs_ctx *ctx, char *ws) {
    GroupedPlan &g = ctx->gp;
    if (g.uploaded_ws == ws) return GBS_OK;
    std::vector<char> &img = ctx->patched_jobs;
    img = ctx->host_jobs;
    for (size_t at : g.relocs) {
        uintptr_t v = 0;
        std::memcpy(&v, img.data() + at, sizeof(v));
        v += reinterpret_cast<uintptr_t>(ws);
        std::memcpy(img.data() + at, &v, sizeof(v));
    }
    HIPCHK(hipMemcpyAsync(ctx->jobs.p, img.data(), img.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    g.uploaded_ws = ws;
    return GBS_OK;
}

// Group-sorted copy of the coil sensitivities (padding slots: 0).
static int build_coil_layout(gbs_ctx *ctx) {
    ctx->coil_l_valid = false;
    if (!ctx->coil_re || !ctx->groups_valid) return GBS_OK;
    const int64_t Kp = ctx->Kpad, K = ctx->K;
    ALLOC(ctx->coil_l, sizeof(float) * 2 * (size_t)ctx->n_coils * (size_t)Kp);
    float *cl = ctx->coil_l.as<float>();
    for (int32_t p = 0; p < ctx->n_coils; ++p) {
        HIPCHK(launch_gather_padded(Kp, ctx->perm.as<int32_t>(), ctx->coil_re + (size_t)p * K, cl + (size_t)(2 * p) * Kp,
                                    ctx->stream));
        HIPCHK(launch_gather_padded(Kp, ctx->perm.as<int32_t>(), ctx->coil_im + (size_t)p * K,
                                    cl + (size_t)(2 * p + 1) * Kp, ctx->stream));
    }
    ctx->coil_l_valid = true;
    return GBS_OK;
}

static int run_grouped(gbs_ctx *ctx, char *ws, const float *m_init, float *m_out, double *sig_out, bool profile,
                       bool use_surr, gbs_stats *st, int *n_timed) {
    const int64_t K = ctx->K;
    const HostSeq &s = ctx->seq;
    if (!ctx->gp.valid) return fail(ctx, GBS_E_STATE, "no grouped schedule (a setter failed)");
    if (int rc = relocate_jobs(ctx, ws)) return rc;
    const GroupedPlan &g = ctx->gp;
    const Plan &plan = g.plan;
    const bool zbuilt = g.zbuilt;
    const int grid = plain_grid(ctx->Kint);
    const bool surr = use_surr && g.surr_rf >= 0;
    char *tb = ws + g.w_tabs;
    char *jb = ctx->jobs.as<char>();
    ctx->partial = g.w_partial ? (double2 *)(ws + g.w_partial) : nullptr;

    // ---- prepare: combined transitions (Eq. 7) and map tables --------------
    // The compositions and folds run on this stream.  The group sums' clearing
    // and the map tables (which depend on the group table alone) run beside
    // them on the side stream, which first waits for everything enqueued here
    // before this point (a previous call's sweeps read the same buffers).  The
    // side stream's kernels are submitted after the compositions, so that the
    // compositions' few workgroups are placed first.
    HIPCHK(hipEventRecord(ctx->fork, ctx->stream));
    if (surr) {
        // network transitions for every z group, exact ones for the checked groups,
        // then exact for all groups only if the check failed (gated on the device)
        char *sb = ws + g.w_surr;
        const gbs_mlp *m = ctx->mlp;
        float *tuples = (float *)(sb + g.s_tuples), *T32 = (float *)(sb + g.s_T32);
        const int32_t *cidx = ctx->surr_idx.as<int32_t>();
        int32_t *fb = (int32_t *)(sb + g.s_fb);
        double *T64 = (double *)(tb + g.rf_off[g.surr_rf]);
        HIPCHK(launch_surr_tuples(ctx->gtab[2].as<float4>(), g.surr_groups, kGammaBar * m->g_ref, tuples,
                                  ctx->stream));
        HIPCHK(mlp_infer_async(m, tuples, nullptr, g.surr_groups, T32, ctx->stream));
        HIPCHK(launch_surr_store(T32, g.surr_groups, T64, ctx->stream));
        HIPCHK(mlp_exact_async(m, tuples, cidx, g.surr_n_check, nullptr, (double *)(sb + g.s_exact), ctx->stream));
        HIPCHK(launch_surr_check(T32, cidx, (const double *)(sb + g.s_exact), g.surr_n_check, ctx->surr_tol,
                                 (float *)(sb + g.s_res), fb, ctx->stream));
        HIPCHK(mlp_exact_async(m, tuples, nullptr, g.surr_groups, fb, T64, ctx->stream));
    }
    HIPCHK(launch_compose((const RfJobDev *)(jb + (surr ? g.o_rf_surr : g.o_rf)), g.n_rf, g.max_rf_groups, s.dt,
                          ctx->stream));
    HIPCHK(hipStreamWaitEvent(ctx->side, ctx->fork, 0));
    HIPCHK(launch_fill_f64((double *)(ws + g.w_gsum), 2 * (int64_t)g.gsum_count, ctx->side));
    HIPCHK(launch_tables((const TabJob *)(jb + g.o_tab), g.n_tab, (int)g.max_tab, ctx->gtab[0].as<float4>(),
                         zbuilt ? ctx->gtab[2].as<float4>() : nullptr, ctx->side));
    HIPCHK(hipEventRecord(ctx->join, ctx->side));
    for (const auto &pj : g.pair_jobs) {
        const RfJob &r = plan.rf[pj.second];
        HIPCHK(launch_compose_pair(ctx->n_runs, ctx->rtab.as<float4>(), ctx->rz.as<float>(),
                                   ctx->d_wave.as<StepW>() + r.step_offset, (int32_t)r.n_steps, s.dt,
                                   (double *)(tb + pj.first), ctx->stream));
    }
    for (const auto &e : g.expand)
        HIPCHK(launch_expand_rows((const double *)(tb + e.first), ctx->tmap.as<int32_t>(), ctx->ng[0],
                                  (double *)(tb + e.second), ctx->stream));
    HIPCHK(launch_fold((const FoldJob *)(jb + g.o_fold), g.n_fold, g.max_fold_groups, ctx->stream));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->join, 0));  // cleared group sums, map tables
    if (st) HIPCHK(hipEventRecord(ctx->ev[1], ctx->stream));

    // ---- sweeps of grouped ops (plain stepping between them) ----------------
    float *mx = (float *)(ws + g.w_state), *my = mx + ctx->Kpad, *mz = my + ctx->Kpad;
    float4 *m_final = (float4 *)(mz + ctx->Kpad);
    const int64_t Kint = ctx->Kint;
    // the default initial state (0, 0, M0) is made by the first sweep itself
    const bool fresh = !m_init && !g.exec.empty() && g.exec.front().first == 0;
    // the fast sweeps hold M / M0: an initial state that gives an isochromat
    // with M0 = 0 a magnetization takes the general sweep instead
    int force_general = 0;
    if (m_init) {
        HIPCHK(launch_fill_f64(ctx->flag.as<double>(), 1, ctx->stream));
        HIPCHK(launch_check_zero_m0(K, ctx->ph.m0, m_init, m_init + K, m_init + 2 * K, ctx->flag.as<int>(), ctx->stream));
        HIPCHK(hipMemcpyAsync(&force_general, ctx->flag.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    if (!fresh)
        HIPCHK(launch_init_state(Kint, ctx->Kpad, ctx->perm.as<int32_t>(), m_init, m_init ? m_init + K : nullptr,
                                 m_init ? m_init + 2 * K : nullptr, ctx->m0i.as<float>(), mx, my, mz, ctx->stream));
    SweepArgs base{};
    base.n4 = Kint / 4;
    base.mx = (float4 *)mx;
    base.my = (float4 *)my;
    base.mz = (float4 *)mz;
    base.m0 = ctx->m0i.as<float4>();
    base.gid_x = ctx->gid[0].as<int4>();
    base.gid_y = ctx->gid[1].as<int4>();
    base.gid_z = ctx->gid[2].as<int4>();
    base.yv = ctx->yi.as<float4>();
    base.zv = ctx->zi.as<float4>();
    base.run_of4 = ctx->run_of4.as<int32_t>();
    const PhantomPtrs iph{ctx->xi.as<float>(), ctx->yi.as<float>(), ctx->zi.as<float>(), ctx->t1i.as<float>(),
                          ctx->t2i.as<float>(), ctx->dfi.as<float>(), ctx->m0i.as<float>()};
    if (ctx->coil_re) {  // sensitivities in layout order (padding slots: 0)
        if (!ctx->coil_l_valid) return fail(ctx, GBS_E_STATE, "no group-sorted coil sensitivities (a setter failed)");
        base.coil = ctx->coil_l.as<float4>();
        base.n_coils = ctx->n_coils;
        base.coil_plane = ctx->Kpad / 4;
    }
    int timed = 0;
    double bytes = 0.0, flops = 0.0;
    const SweepOp *dev_ops = (const SweepOp *)(jb + g.o_sweep);
    // a run that ends with a state-writing sweep leaves its state in m_final
    const bool final4 = !g.exec.empty() && g.exec.back().first == 0 && g.segs[g.exec.back().second].write_m;
    for (size_t e = 0; e < g.exec.size(); ++e) {
        const auto &item = g.exec[e];
        if (item.first == 0) {
            const GroupedPlan::Seg &sg = g.segs[item.second];
            SweepArgs a = base;
            a.ops = dev_ops + sg.op_begin;
            a.n_ops = sg.op_end - sg.op_begin;
            a.need = sg.need | (force_general ? kForceGeneral : 0);
            a.write_m = sg.write_m ? 1 : 0;
            a.m_final = (final4 && e + 1 == g.exec.size()) ? m_final : nullptr;
            a.fresh = (fresh && e == 0) ? 1 : 0;
            a.n_head = sg.n_head;
            if (a.m_final || a.fresh) {  // the whole state is written, so all of it is held
                a.need |= kNeedMz;
                a.write_m = 1;
            }
            bytes += sweep_bytes_per_iso(a.need, a.write_m != 0, a.fresh != 0, a.m_final != nullptr) * (double)K;
            flops += sg.flops_per_iso * (double)K;
            if (profile) HIPCHK(hipEventRecord(ctx->pev[2 * timed], ctx->stream));
            HIPCHK(launch_sweep(a, ctx->stream));
            if ((a.need & kPartials) && in_partial_kernel(a.need, a.coil != nullptr)) {  // (else atomics were used)
                const auto &sp = g.seg_parts[item.second];
                HIPCHK(launch_part_reduce((const PartJob *)(jb + g.o_part) + sp.first, sp.second, ctx->ng[0],
                                          ctx->xstart.as<int32_t>(), ctx->stream));
            }
            if (profile) HIPCHK(hipEventRecord(ctx->pev[2 * timed++ + 1], ctx->stream));
        } else {
            const Op &op = plan.ops[item.second];
            PlainArgs a = step_args(ctx, op.step, iph, Kint, mx, my, mz, mx, my, mz);
            const bool b1 = op.step.block >= 0 && ctx->cls[op.step.block].has_b1;
            const int64_t s0 = op.step.block >= 0 ? s.blocks[op.step.block].sample_offset + op.step.sample_lo : 0;
            const float *cl = ctx->coil_re ? ctx->coil_l.as<float>() : nullptr;  // planes re, im per coil
            const int64_t Kp = ctx->Kpad;
            if (int rc = launch_steps(ctx, a, b1, grid, cl, cl ? cl + Kp : nullptr, 2 * Kp, sig_out, s0))
                return rc;
        }
    }
    *n_timed = timed;
    if (st) HIPCHK(hipEventRecord(ctx->ev[2], ctx->stream));

    // ---- final state into the caller's order, on the side stream ------------
    HIPCHK(hipEventRecord(ctx->fork, ctx->stream));
    HIPCHK(hipStreamWaitEvent(ctx->side, ctx->fork, 0));
    if (final4)
        HIPCHK(launch_gather_state4(K, ctx->inv.as<int32_t>(), m_final, m_out, m_out + K, m_out + 2 * K, ctx->side));
    else
        HIPCHK(launch_gather_state(K, ctx->inv.as<int32_t>(), mx, my, mz, m_out, m_out + K, m_out + 2 * K,
                                    ctx->side));
    HIPCHK(hipEventRecord(ctx->join, ctx->side));

    // ---- ADC samples from the group sums (Eq. 8, Eq. 10) --------------------
    HIPCHK(launch_adc_eval((const AdcJobDev *)(jb + g.o_adc), g.n_adc, g.max_adc_groups, g.max_adc_samples,
                           sig_out, ctx->stream));
    HIPCHK(launch_adc_lin((const AdcLinJob *)(jb + g.o_adclin), g.n_adclin, g.max_adclin_groups, sig_out,
                          ctx->stream));
    if (st) HIPCHK(hipEventRecord(ctx->ev[3], ctx->stream));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->join, 0));
    if (st) {
        st->n_passes = g.n_ops;
        st->n_sweeps = (int64_t)g.segs.size();
        st->n_emit_only = plan.n_emit_only;
        st->n_rf_grouped = plan.n_rf_grouped;
        st->n_adc_grouped = plan.n_adc_grouped;
        st->n_fallback = plan.n_fallback;
        st->n_distinct_rf = (int64_t)plan.rf.size();
        st->n_b1zero = plan.n_b1zero;
        st->pass_bytes = bytes;
        st->pass_flops = flops;
    }
    return GBS_OK;
}

// The conventional accelerated method (Sec. 2.2): per-isochromat combined
// transitions with dynamic caching, direct evaluation of with-ADC blocks.
// The state lives in FP64 (state64) from the first operation that writes it;
// until then operations read m_init or (0, 0, M0).  The last operation always
// writes m_out.
// Cached schedule: host plan, per-sample tables of the direct ADC operations
// on the device, GBS_PROFILE events.
static int build_cached_surrogate(gbs_ctx *ctx);

static int build_cached_plan(gbs_ctx *ctx) {
    const double dt = ctx->seq.dt;
    ctx->cplan_valid = false;
    {
        ctx->cplan = plan_cached(ctx->seq, ctx->cls, step_samples(ctx));
        const Plan &plan = ctx->cplan;
        // sample n of a direct ADC operation: c_n = gamma_bar (m_pre + m(s_n)),
        // tau_n = tau_pre + s_n dt, with m(s) the block's gradient moment over
        // its first s raster steps
        std::vector<double4> tab;
        ctx->csamp_off.assign(plan.ops.size(), -1);
        int64_t mom_block = -1;
        std::vector<double> mom[3];
        for (size_t oi = 0; oi < plan.ops.size(); ++oi) {
            const Op &op = plan.ops[oi];
            if (op.kind != 3) continue;
            const CachedOp &c = op.cached;
            const gbs_block &b = ctx->seq.blocks[c.block];
            if (c.block != mom_block) {
                const std::vector<float> *g[3] = {&ctx->seq.gx, &ctx->seq.gy, &ctx->seq.gz};
                for (int a = 0; a < 3; ++a) {
                    mom[a].assign((size_t)b.n_steps + 1, 0.0);
                    for (int64_t j = 0; j < b.n_steps; ++j)
                        mom[a][j + 1] = mom[a][j] + (double)(*g[a])[b.step_offset + j] * dt;
                }
                mom_block = c.block;
            }
            ctx->csamp_off[oi] = (int64_t)tab.size();
            for (int32_t n = c.sample_lo; n < c.sample_hi; ++n) {
                const int32_t sn = ctx->seq.adc_idx[b.sample_offset + n];
                tab.push_back(make_double4(kGammaBar * (c.pre.m[0] + mom[0][sn]), kGammaBar * (c.pre.m[1] + mom[1][sn]),
                                           kGammaBar * (c.pre.m[2] + mom[2][sn]), c.pre.tau + (double)sn * dt));
            }
        }
        ALLOC(ctx->csamp, sizeof(double4) * std::max<size_t>(tab.size(), 1));
        if (!tab.empty())
            HIPCHK(hipMemcpy(ctx->csamp.p, tab.data(), sizeof(double4) * tab.size(), hipMemcpyHostToDevice));
    }
    while (ctx->pev.size() < 2 * ctx->cplan.ops.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        ctx->pev.push_back(e);
    }
    ctx->cplan_valid = true;
    return build_cached_surrogate(ctx);
}

// GBS_CACHED with the surrogate: the first cache entry whose waveform is the
// network's pulse, and n_check distinct seeded isochromats for its spot check.
static int build_cached_surrogate(gbs_ctx *ctx) {
    ctx->csurr_entry = -1;
    ctx->csurr_n_check = 0;
    if (!ctx->mlp || !ctx->cplan_valid || ctx->K <= 0) return GBS_OK;
    const Plan &plan = ctx->cplan;
    for (size_t i = 0; i < plan.rf.size(); ++i)
        if (matches_pulse(ctx, plan.rf[i].step_offset, plan.rf[i].n_steps)) {
            ctx->csurr_entry = (int)i;
            break;
        }
    if (ctx->csurr_entry < 0) return GBS_OK;
    const int64_t K = ctx->K;
    const int32_t n = (int32_t)std::min<int64_t>(ctx->surr_check, K);
    std::vector<int32_t> idx;
    std::unordered_set<int64_t> seen;
    uint64_t rs = ctx->surr_seed ^ 0x2545F4914F6CDD1Dull;
    while ((int32_t)idx.size() < n) {  // distinct draws from [0, K)
        rs = rs * 6364136223846793005ull + 1442695040888963407ull;
        const int64_t k = (int64_t)((rs >> 17) % (uint64_t)K);
        if (seen.insert(k).second) idx.push_back((int32_t)k);
    }
    ALLOC(ctx->csurr_idx, sizeof(int32_t) * (size_t)n);
    HIPCHK(hipMemcpy(ctx->csurr_idx.p, idx.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
    ctx->csurr_n_check = n;
    return GBS_OK;
}

// Workspace of GBS_CACHED: the FP64 state, the transition cache (3 float4
// rows of K per distinct with-RF waveform), per-workgroup sample sums and,
// with an attached surrogate whose pulse the sequence plays, its spot-check
// tuples, exact transitions, residual and fallback flag.
struct CachedWs {
    size_t state = 0, cache = 0, partial = 0, s_tuples = 0, s_exact = 0, s_res = 0, s_fb = 0;
};

static size_t cached_ws(const gbs_ctx *ctx, CachedWs *o) {
    const int64_t K = ctx->K;
    const size_t n_entries = ctx->cplan.rf.size();
    WsCarve w;
    o->state = w.take(sizeof(double) * 3 * (size_t)K);
    o->cache = n_entries ? w.take(sizeof(float4) * 3 * (size_t)K * n_entries) : 0;
    const int pgrid = plain_grid(K), agrid = direct_adc_grid(K);
    o->partial = w.take(sizeof(double2) * (size_t)std::max(pgrid, agrid) * kMaxSamplesPerLaunch * (size_t)ctx->n_coils);
    if (ctx->csurr_entry >= 0) {
        o->s_tuples = w.take(sizeof(float) * 5 * (size_t)ctx->csurr_n_check);
        o->s_exact = w.take(sizeof(double) * 12 * (size_t)ctx->csurr_n_check);
        o->s_res = w.take(sizeof(float));
        o->s_fb = w.take(sizeof(int32_t));
    }
    return w.off;
}

static int run_cached(gbs_ctx *ctx, char *ws, const float *m_init, float *m_out, double *sig_out, bool profile,
                      bool use_surr, gbs_stats *st, int *n_timed) {
    const int64_t K = ctx->K;
    const double dt = ctx->seq.dt;
    if (!ctx->cplan_valid) return fail(ctx, GBS_E_STATE, "no cached schedule (a setter failed)");
    const Plan &plan = ctx->cplan;
    const size_t n_entries = plan.rf.size();
    CachedWs o;
    cached_ws(ctx, &o);
    const int pgrid = plain_grid(K), agrid = direct_adc_grid(K);
    ctx->partial = (double2 *)(ws + o.partial);
    float4 *cache = (float4 *)(ws + o.cache);
    ctx->cprof_kind.clear();
    double *s64 = (double *)(ws + o.state);
    const bool surr = use_surr && ctx->csurr_entry >= 0;
    const float *mi_x = m_init, *mi_y = m_init ? m_init + K : nullptr, *mi_z = m_init ? m_init + 2 * K : nullptr;
    bool from_init = true;
    int timed = 0;
    for (size_t oi = 0; oi < plan.ops.size(); ++oi) {
        const Op &op = plan.ops[oi];
        if (profile) HIPCHK(hipEventRecord(ctx->pev[2 * timed], ctx->stream));
        if (op.kind == 1) {  // RF during ADC: plain FP64 stepping
            PlainArgs a = step_args(ctx, op.step, ctx->ph, K, from_init ? mi_x : nullptr, from_init ? mi_y : nullptr,
                                    from_init ? mi_z : nullptr, nullptr, nullptr, nullptr);
            if (!from_init) {
                a.min64_x = s64;
                a.min64_y = s64 + K;
                a.min64_z = s64 + 2 * K;
            }
            a.mout64_x = s64;
            a.mout64_y = s64 + K;
            a.mout64_z = s64 + 2 * K;
            const int64_t s0 = ctx->seq.blocks[op.step.block].sample_offset + op.step.sample_lo;
            if (int rc = launch_steps(ctx, a, ctx->cls[op.step.block].has_b1, pgrid, ctx->coil_re, ctx->coil_im,
                                      K, sig_out, s0))
                return rc;
            from_init = false;
        } else if (op.kind == 3) {  // direct ADC: reads the state, writes samples
            const CachedOp &c = op.cached;
            const gbs_block &b = ctx->seq.blocks[c.block];
            DirectAdcArgs a{};
            a.K = K;
            a.ph = ctx->ph;
            if (from_init) {
                a.min_x = mi_x;
                a.min_y = mi_y;
            } else {
                a.s64_in = s64;
            }
            a.samp = ctx->csamp.as<double4>() + ctx->csamp_off[oi];
            a.n_samples = c.sample_hi - c.sample_lo;
            a.partial = ctx->partial;
            a.coil_re = ctx->coil_re;
            a.coil_im = ctx->coil_im;
            a.n_coils = ctx->coil_re ? ctx->n_coils : 1;
            HIPCHK(launch_direct_adc(a, agrid, ctx->stream));
            for (int32_t p = 0; p < a.n_coils; ++p)  // partials of coil p: [grid][n_samples] block p
                HIPCHK(launch_plain_finalize(
                    ctx->partial + (size_t)p * agrid * a.n_samples, agrid, a.n_samples,
                    sig_out + 2 * ((int64_t)p * ctx->seq.total_samples + b.sample_offset + c.sample_lo), ctx->stream));
        } else {  // 2: cached transition (composed at first use); 4: final map
            const CachedOp &c = op.cached;
            CachedArgs a{};
            a.K = K;
            a.ph = ctx->ph;
            if (from_init) {
                a.min_x = mi_x;
                a.min_y = mi_y;
                a.min_z = mi_z;
            } else {
                a.s64_in = s64;
            }
            if (op.kind == 4) {
                a.mout_x = m_out;
                a.mout_y = m_out + K;
                a.mout_z = m_out + 2 * K;
            } else {
                a.s64_out = s64;
            }
            a.has_pre = c.has_pre ? 1 : 0;
            a.pre_tau = c.pre.tau;
            for (int i = 0; i < 3; ++i) a.pre_cyc[i] = kGammaBar * c.pre.m[i];
            a.dt = dt;
            a.gdt = kTwoPi * kGammaBar * dt;
            int mode = kCacheMap;
            if (op.kind == 2) {
                const gbs_block &b = ctx->seq.blocks[c.block];
                a.cache = cache + 3 * (size_t)K * (size_t)c.entry;
                mode = c.compose ? kCacheCompose : kCacheApply;
                a.wave = ctx->d_wave.as<StepW>() + b.step_offset;
                a.n_steps = (int32_t)b.n_steps;
            }
            if (mode == kCacheCompose && surr && c.entry == ctx->csurr_entry) {
                // the network fills the entry for every isochromat; n_check of
                // them are composed exactly and compared; past tol the exact
                // composition runs after all (compose launch gated on the
                // flag), else the network's entry is applied
                const gbs_mlp *m = ctx->mlp;
                float *tup = (float *)(ws + o.s_tuples);
                double *ex = (double *)(ws + o.s_exact);
                int32_t *fb = (int32_t *)(ws + o.s_fb);
                const int32_t *cidx = ctx->csurr_idx.as<int32_t>();
                HIPCHK(mlp_infer_rows_async(m, ctx->ph.z, ctx->ph.df, ctx->ph.t1, ctx->ph.t2, K, a.cache, K,
                                            ctx->stream));
                HIPCHK(launch_surr_iso_tuples(ctx->ph.z, ctx->ph.df, ctx->ph.t1, ctx->ph.t2, cidx, ctx->csurr_n_check,
                                              kGammaBar * m->g_ref, tup, ctx->stream));
                HIPCHK(mlp_exact_async(m, tup, nullptr, ctx->csurr_n_check, nullptr, ex, ctx->stream));
                HIPCHK(launch_surr_check_rows(a.cache, K, cidx, ex, ctx->csurr_n_check, ctx->surr_tol,
                                              (float *)(ws + o.s_res), fb, ctx->stream));
                a.gate = fb;
                a.gate_value = 1;
                HIPCHK(launch_cached(a, kCacheCompose, ctx->stream));
                a.gate_value = 0;
                HIPCHK(launch_cached(a, kCacheApply, ctx->stream));
            } else {
                HIPCHK(launch_cached(a, mode, ctx->stream));
            }
            from_init = false;
        }
        if (profile) {
            HIPCHK(hipEventRecord(ctx->pev[2 * timed + 1], ctx->stream));
            ++timed;
            // 0: compose, 1: cached transition or map, 2: direct ADC, 3: stepped
            ctx->cprof_kind.push_back(op.kind == 1 ? 3 : op.kind == 3 ? 2 : (op.kind == 2 && op.cached.compose) ? 0 : 1);
        }
    }
    *n_timed = timed;
    if (st) {
        st->n_rf_cached = plan.n_rf_cached;
        st->n_adc_direct = plan.n_adc_direct;
        st->n_fallback = plan.n_fallback;
        st->n_distinct_rf = (int64_t)n_entries;
        st->n_b1zero = plan.n_b1zero;
        st->cache_bytes = (double)(sizeof(float4) * 3 * (size_t)K * n_entries);
    }
    return GBS_OK;
}

// The schedules of every mode for the current phantom, sequence, groups,
// coils and surrogate: built by the setters, so that gbs_simulate allocates
// nothing.  Plain and cached schedules need a sequence; the grouped one also
// valid groups.
static int refresh_plans(gbs_ctx *ctx) {
    ctx->pplan_valid = ctx->cplan_valid = false;
    ctx->gp.valid = false;
    if (!ctx->has_seq) return GBS_OK;
    build_plain_plan(ctx);
    if (int rc = build_cached_plan(ctx)) return rc;
    if (!ctx->groups_valid) return GBS_OK;
    if (int rc = build_coil_layout(ctx)) return rc;
    return build_grouped_plan(ctx);
}

// Workspace bytes of `mode` for the current schedules (0 if the mode needs
// none); -1 with the message set when the mode cannot run yet.
static int workspace_bytes(gbs_ctx *ctx, int mode, size_t *bytes) {
    if (!ctx->has_ph) return fail(ctx, GBS_E_STATE, "no phantom (gbs_set_phantom)");
    if (!ctx->has_seq) return fail(ctx, GBS_E_STATE, "no sequence (gbs_set_sequence)");
    if (mode != GBS_PLAIN && mode != GBS_GROUPED && mode != GBS_CACHED)
        return fail(ctx, GBS_E_INVALID, "mode must be GBS_PLAIN, GBS_GROUPED or GBS_CACHED");
    size_t a = 0, b = 0;
    if (mode == GBS_PLAIN) {
        if (!ctx->pplan_valid) return fail(ctx, GBS_E_STATE, "no plain schedule (a setter failed)");
        *bytes = plain_ws(ctx, &a, &b);
    } else if (mode == GBS_CACHED) {
        if (!ctx->cplan_valid) return fail(ctx, GBS_E_STATE, "no cached schedule (a setter failed)");
        CachedWs o;
        *bytes = cached_ws(ctx, &o);
    } else {
        if (!ctx->groups_valid) return fail(ctx, GBS_E_STATE, "GBS_GROUPED needs gbs_build_groups on the current phantom");
        if (!ctx->gp.valid) return fail(ctx, GBS_E_STATE, "no grouped schedule (a setter failed)");
        *bytes = ctx->gp.ws_bytes;
    }
    return GBS_OK;
}

extern "C" int gbs_workspace_size(gbs_ctx *ctx, int mode, size_t *bytes) {
    if (!ctx) return GBS_E_INVALID;
    if (!bytes) return fail(ctx, GBS_E_INVALID, "null bytes");
    *bytes = 0;
    return workspace_bytes(ctx, mode, bytes);
}

extern "C" int gbs_simulate(gbs_ctx *ctx, int mode, uint32_t flags, void *workspace, size_t ws_bytes,
                            const float *m_init, float *m_out, double *sig_out, gbs_stats *stats) {
    if (!ctx) return GBS_E_INVALID;
    if (!ctx->has_ph) return fail(ctx, GBS_E_STATE, "gbs_simulate before gbs_set_phantom");
    if (!ctx->has_seq) return fail(ctx, GBS_E_STATE, "gbs_simulate before gbs_set_sequence");
    if (mode != GBS_PLAIN && mode != GBS_GROUPED && mode != GBS_CACHED)
        return fail(ctx, GBS_E_INVALID, "mode must be GBS_PLAIN, GBS_GROUPED or GBS_CACHED");
    if (!m_out || (ctx->seq.total_samples > 0 && !sig_out)) return fail(ctx, GBS_E_INVALID, "null output");
    if (mode == GBS_GROUPED && !ctx->groups_valid)
        return fail(ctx, GBS_E_STATE, "GBS_GROUPED needs gbs_build_groups on the current phantom");
    if (flags & ~(GBS_ASYNC | GBS_PROFILE | GBS_SURROGATE))
        return fail(ctx, GBS_E_INVALID, "unknown flags");
    const bool use_surr = (flags & GBS_SURROGATE) != 0;
    if (use_surr && (mode == GBS_PLAIN || !ctx->mlp))
        return fail(ctx, GBS_E_INVALID, "GBS_SURROGATE needs GBS_GROUPED or GBS_CACHED and gbs_set_surrogate");
    size_t need = 0;
    if (int rc = workspace_bytes(ctx, mode, &need)) return rc;
    if (!workspace || ws_bytes < need)
        return fail(ctx, GBS_E_WORKSPACE, "workspace of " + std::to_string(workspace ? ws_bytes : 0) +
                                              " bytes; this mode needs " + std::to_string(need) +
                                              " (gbs_workspace_size)");
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return fail(ctx, GBS_E_WORKSPACE, "workspace must be 256-byte aligned");
    char *ws = static_cast<char *>(workspace);
    HIPCHK(hipSetDevice(ctx->device));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        HIPCHK(hipEventRecord(ctx->ev[0], ctx->stream));
    }
    if (ctx->seq.total_samples > 0)
        HIPCHK(launch_fill_f64(sig_out, 2 * (int64_t)ctx->n_coils * ctx->seq.total_samples, ctx->stream));
    const bool profile = (flags & GBS_PROFILE) != 0;
    int n_timed = 0;
    int rc = mode == GBS_PLAIN ? run_plain(ctx, ws, m_init, m_out, sig_out, stats)
             : mode == GBS_CACHED ? run_cached(ctx, ws, m_init, m_out, sig_out, profile, use_surr, stats, &n_timed)
                                  : run_grouped(ctx, ws, m_init, m_out, sig_out, profile, use_surr, stats, &n_timed);
    if (rc != GBS_OK) return rc;
    if (stats) HIPCHK(hipEventRecord(ctx->ev[4], ctx->stream));
    if (!(flags & GBS_ASYNC) || stats || profile) {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        HIPCHK(hipGetLastError());
    }
    if (stats) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[4]));
        stats->ms_total = ms;
        if (mode == GBS_PLAIN) {
            stats->ms_stepped = ms;
        } else if (mode == GBS_CACHED) {
            double sum[4] = {0.0, 0.0, 0.0, 0.0};
            for (int i = 0; i < n_timed; ++i) {
                HIPCHK(hipEventElapsedTime(&ms, ctx->pev[2 * i], ctx->pev[2 * i + 1]));
                sum[ctx->cprof_kind[i]] += ms;
            }
            stats->ms_compose = sum[0];
            stats->ms_apply = sum[1];
            stats->ms_adc_direct = sum[2];
            stats->ms_stepped = sum[3];
            if (use_surr && ctx->csurr_entry >= 0) {
                CachedWs o;
                cached_ws(ctx, &o);
                float res = 0.f;
                int32_t fb = 0;
                HIPCHK(hipMemcpyAsync(&res, ws + o.s_res, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
                HIPCHK(hipMemcpyAsync(&fb, ws + o.s_fb, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
                HIPCHK(hipStreamSynchronize(ctx->stream));
                stats->n_surrogate = 1;
                stats->n_surrogate_fallback = fb ? 1 : 0;
                stats->surrogate_residual = res;
            }
        } else {
            HIPCHK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
            stats->ms_prepare = ms;
            HIPCHK(hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]));
            stats->ms_passes = ms;
            HIPCHK(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]));
            stats->ms_adc_eval = ms;
            double sum = 0.0;
            for (int i = 0; i < n_timed; ++i) {
                HIPCHK(hipEventElapsedTime(&ms, ctx->pev[2 * i], ctx->pev[2 * i + 1]));
                sum += ms;
            }
            stats->pass_kernel_ms = sum;
            const GroupedPlan &g = ctx->gp;
            if (use_surr && g.surr_rf >= 0) {
                float res = 0.f;
                int32_t fb = 0;
                const char *sb = ws + g.w_surr;
                HIPCHK(hipMemcpyAsync(&res, sb + g.s_res, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
                HIPCHK(hipMemcpyAsync(&fb, sb + g.s_fb, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
                HIPCHK(hipStreamSynchronize(ctx->stream));
                stats->n_surrogate = 1;
                stats->n_surrogate_fallback = fb ? 1 : 0;
                stats->surrogate_residual = res;
            }
        }
    }
    return GBS_OK;
}

extern "C" int gbs_set_surrogate(gbs_ctx *ctx, gbs_mlp *m, float tol, int32_t n_check, uint64_t seed) {
    if (!ctx) return GBS_E_INVALID;
    if (m) {
        if (!(tol > 0.f) || !std::isfinite(tol)) return fail(ctx, GBS_E_INVALID, "tol must be positive");
        if (n_check < 1) return fail(ctx, GBS_E_INVALID, "n_check must be >= 1");
        if (m->device != ctx->device) return fail(ctx, GBS_E_INVALID, "network lives on another device");
        if (!m->has_pulse) return fail(ctx, GBS_E_STATE, "network has no pulse (gbs_mlp_set_pulse)");
    }
    ctx->mlp = m;
    ctx->surr_tol = tol;
    ctx->surr_check = n_check;
    ctx->surr_seed = seed;
    ctx->gp.valid = false;
    HIPCHK(hipSetDevice(ctx->device));
    if (int rc = build_cached_surrogate(ctx)) return rc;
    if (ctx->has_seq && ctx->groups_valid) return build_grouped_plan(ctx);
    return GBS_OK;
}

// ------------------------------------------------------------------ adjoint
extern "C" int gbs_adj_forward(gbs_ctx *ctx, const int32_t *cls, int32_t n_classes, const float *t1c,
                               const float *t2c, const float *rf_param, int64_t n_rf, const int32_t *param_blocks,
                               int32_t n_param_blocks, int32_t every, double *sig_out) {
    if (!ctx) return GBS_E_INVALID;
    ctx->adj_ready = false;
    if (!ctx->has_ph) return fail(ctx, GBS_E_STATE, "gbs_adj_forward before gbs_set_phantom");
    if (!ctx->has_seq) return fail(ctx, GBS_E_STATE, "gbs_adj_forward before gbs_set_sequence");
    if (!cls || !t1c || !t2c || !rf_param || (ctx->seq.total_samples > 0 && !sig_out))
        return fail(ctx, GBS_E_INVALID, "null argument");
    if (n_classes < 1 || n_classes > kAdjMaxClasses)
        return fail(ctx, GBS_E_INVALID, "n_classes must be in [1, 64]");
    if (n_rf < 1 || n_rf > kAdjMaxRf) return fail(ctx, GBS_E_INVALID, "n_rf must be in [1, 3072]");
    if (every < kAdjSub || every > kAdjMaxEvery || every % kAdjSub)
        return fail(ctx, GBS_E_INVALID, "checkpoint interval must be a multiple of 8 in [8, 256]");
    if (n_param_blocks < 0 || (n_param_blocks > 0 && !param_blocks))
        return fail(ctx, GBS_E_INVALID, "bad parameter block list");
    const HostSeq &s = ctx->seq;
    const int64_t nb = (int64_t)s.blocks.size();
    std::vector<char> is_par(nb, 0);
    for (int32_t i = 0; i < n_param_blocks; ++i) {
        const int32_t b = param_blocks[i];
        if (b < 0 || b >= nb || s.blocks[b].type != GBS_BLOCK_RF || s.blocks[b].n_steps != n_rf)
            return fail(ctx, GBS_E_INVALID, "parameter blocks must be RF blocks of n_rf steps");
        is_par[b] = 1;
    }
    // Flatten the sequence into ops: a relaxation block is one op (Eq. 4, 5);
    // raster steps of a parameter block, or with B1 != 0, are one op each
    // (Eq. 2, A1, A2); every other run of raster steps without RF between
    // two sample boundaries is one op too, the closed form of Eq. 4, 5 with
    // the run's gradient moment summed in FP64 (with B1 = 0 every step is a
    // z rotation, so the run's product is exactly that closed form, and its
    // phase is formed in FP64 once instead of rounded at every step).
    std::vector<AdjOp> ops;
    std::vector<int32_t> spos((size_t)s.total_samples);
    std::vector<int64_t> bop;  // op boundary of each raster boundary of the current block
    for (int64_t b = 0; b < nb; ++b) {
        const gbs_block &bk = s.blocks[b];
        if (bk.type == GBS_BLOCK_RELAX) {
            AdjOp op{};
            op.kind = 1;
            op.param = -1;
            op.tau = bk.tau;
            for (int i = 0; i < 3; ++i) op.cyc[i] = kGammaBar * bk.moment[i];
            ops.push_back(op);
            continue;
        }
        std::vector<char> cut((size_t)bk.n_steps + 1, 0);  // a sample is taken at this raster boundary
        for (int32_t n = 0; n < bk.n_samples; ++n) cut[(size_t)s.adc_idx[bk.sample_offset + n]] = 1;
        bop.assign((size_t)bk.n_steps + 1, -1);
        int64_t j = 0;
        while (j < bk.n_steps) {
            const size_t w0 = (size_t)(bk.step_offset + j);
            bop[(size_t)j] = (int64_t)ops.size();
            AdjOp op{};
            op.param = -1;
            if (!is_par[b] && s.rf_re[w0] == 0.f && s.rf_im[w0] == 0.f) {
                double mom[3] = {0.0, 0.0, 0.0};
                const int64_t j0 = j;
                do {
                    const size_t w = (size_t)(bk.step_offset + j);
                    mom[0] += (double)s.gx[w] * s.dt;
                    mom[1] += (double)s.gy[w] * s.dt;
                    mom[2] += (double)s.gz[w] * s.dt;
                    ++j;
                } while (j < bk.n_steps && !cut[(size_t)j] && s.rf_re[bk.step_offset + j] == 0.f &&
                         s.rf_im[bk.step_offset + j] == 0.f);
                op.kind = 1;
                op.tau = (double)(j - j0) * s.dt;
                for (int i = 0; i < 3; ++i) op.cyc[i] = kGammaBar * mom[i];
            } else {
                op.kind = 0;
                op.b1r = s.rf_re[w0];
                op.b1i = s.rf_im[w0];
                op.gx = s.gx[w0];
                op.gy = s.gy[w0];
                op.gz = s.gz[w0];
                op.param = is_par[b] ? (int32_t)j : -1;
                ++j;
            }
            ops.push_back(op);
        }
        bop[(size_t)bk.n_steps] = (int64_t)ops.size();
        for (int32_t n = 0; n < bk.n_samples; ++n)
            spos[bk.sample_offset + n] = (int32_t)bop[(size_t)s.adc_idx[bk.sample_offset + n]];
    }
    const int64_t n_ops = (int64_t)ops.size();
    if (n_ops > (int64_t)INT32_MAX - 2) return fail(ctx, GBS_E_INVALID, "sequence too long for the adjoint");
    const int64_t N = s.total_samples;
    std::vector<int32_t> samp((size_t)(n_ops + 2 + N), 0);  // sstart[n_ops + 2], then sid[N]
    for (int64_t n = 0; n < N; ++n) samp[spos[n] + 1]++;
    for (int64_t p = 0; p <= n_ops; ++p) samp[p + 1] += samp[p];
    {
        std::vector<int32_t> fill((size_t)(n_ops + 1), 0);
        for (int64_t n = 0; n < N; ++n) samp[n_ops + 2 + samp[spos[n]] + fill[spos[n]]++] = (int32_t)n;
    }
    HIPCHK(hipSetDevice(ctx->device));
    const int64_t K = ctx->K;
    const int grid = (int)((K + kAdjWG - 1) / kAdjWG);
    const int64_t n_ckpt = (n_ops + every - 1) / every;
    ALLOC(ctx->adj_ops, sizeof(AdjOp) * (size_t)std::max<int64_t>(n_ops, 1));
    ALLOC(ctx->adj_samp, sizeof(int32_t) * samp.size());
    ALLOC(ctx->adj_ckpt, sizeof(float) * 3 * (size_t)K * (size_t)std::max<int64_t>(n_ckpt, 1));
    ALLOC(ctx->adj_sub, sizeof(float) * 3 * (size_t)K * (size_t)(every / kAdjSub));
    ALLOC(ctx->adj_sig, sizeof(double2) * (size_t)grid * (size_t)std::max<int64_t>(N, 1));
    ALLOC(ctx->adj_grf, sizeof(float2) * (size_t)grid * (size_t)n_rf);
    ALLOC(ctx->adj_gt, sizeof(double2) * (size_t)grid * (size_t)n_classes);
    ALLOC(ctx->flag, 256);
    // inputs: class indices in range, T1/T2 > 0 (checked on the device)
    HIPCHK(launch_fill_f64(ctx->flag.as<double>(), 1, ctx->stream));
    HIPCHK(launch_adj_validate(K, cls, n_classes, t1c, t2c, ctx->flag.as<int>(), ctx->stream));
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, ctx->flag.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (bad) return fail(ctx, GBS_E_INVALID, "class index out of range or T1/T2 <= 0");
    if (n_ops > 0) HIPCHK(hipMemcpy(ctx->adj_ops.p, ops.data(), sizeof(AdjOp) * (size_t)n_ops, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->adj_samp.p, samp.data(), sizeof(int32_t) * samp.size(), hipMemcpyHostToDevice));
    AdjArgs a{};
    a.K = K;
    a.x = ctx->ph.x;
    a.y = ctx->ph.y;
    a.z = ctx->ph.z;
    a.df = ctx->ph.df;
    a.m0 = ctx->ph.m0;
    a.cls = cls;
    a.t1c = t1c;
    a.t2c = t2c;
    a.n_classes = n_classes;
    a.ops = ctx->adj_ops.as<AdjOp>();
    a.n_ops = (int32_t)n_ops;
    a.rfp = (const float2 *)rf_param;
    a.n_rf = (int32_t)n_rf;
    a.sstart = ctx->adj_samp.as<int32_t>();
    a.sid = ctx->adj_samp.as<int32_t>() + n_ops + 2;
    a.dt = s.dt;
    a.every = every;
    a.ckpt = ctx->adj_ckpt.as<float>();
    a.sub = ctx->adj_sub.as<float>();
    a.N = (int32_t)N;
    a.sig_part = ctx->adj_sig.as<double2>();
    a.grf_part = ctx->adj_grf.as<float2>();
    a.gt_part = ctx->adj_gt.as<double2>();
    HIPCHK(launch_adj_forward(a, ctx->stream));
    HIPCHK(launch_adj_finalize(a, sig_out, nullptr, nullptr, nullptr, true, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
    ctx->adj = a;
    ctx->adj_ready = true;
    return GBS_OK;
}

extern "C" int gbs_adj_backward(gbs_ctx *ctx, const double *grad_sig, float *grad_rf, double *grad_t1,
                                double *grad_t2) {
    if (!ctx) return GBS_E_INVALID;
    if (!ctx->adj_ready) return fail(ctx, GBS_E_STATE, "gbs_adj_backward without a preceding gbs_adj_forward");
    if ((ctx->adj.N > 0 && !grad_sig) || !grad_rf || !grad_t1 || !grad_t2)
        return fail(ctx, GBS_E_INVALID, "null argument");
    HIPCHK(hipSetDevice(ctx->device));
    AdjArgs a = ctx->adj;
    a.w = (const double2 *)grad_sig;
    HIPCHK(launch_adj_backward(a, ctx->stream));
    HIPCHK(launch_adj_finalize(a, nullptr, grad_rf, grad_t1, grad_t2, false, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipGetLastError());
    return GBS_OK;
}
