/*
 * gbloch.h -- C ABI of the grouped-isochromat Bloch simulator for gfx950.
 *
 * The library simulates K static isochromats under a block-structured pulse
 * sequence, after H. Takeshima, "Fast Magnetic Resonance Simulation Using
 * Combined Update with Grouped Isochromats":
 *
 *   - per raster step dt every isochromat's homogeneous state
 *     (Mx, My, Mz, M0) is multiplied by U = D R (Eq. 2; Appendix A, Eq. A1
 *     and Eq. A2): R rotates about u = B/|B| by theta = -gamma |B| dt with
 *     B = (Re B1, Im B1, G . r + dB0) held constant over the step, D applies
 *     T2 decay and T1 recovery toward M0;
 *   - relaxation blocks (no RF, no ADC) use the closed forms Eq. (4), (5);
 *   - ADC sample n adds Mx + i My of all isochromats at its raster boundary
 *     (Eq. 6): one receive coil of unit sensitivity, or P coils with
 *     per-isochromat sensitivities S(k, p) (gbs_set_coils);
 *   - GBS_PLAIN steps every isochromat individually (the conventional
 *     method, Sec. 2.2); GBS_GROUPED uses the paper's combined update with
 *     grouped isochromats (Sec. 2.3, 2.4): isochromats sharing
 *     (r_a, T1, T2, dB0) share one combined transition T (Eq. 7) for an
 *     a-only subsequence, and with-ADC subsequences evolve per-group sums
 *     (Eq. 8-10) instead of every member;
 *   - GBS_CACHED is the conventional accelerated method of Sec. 2.2 that the
 *     grouped update is compared with: every isochromat gets its own combined
 *     transition T_k (Eq. 7) per distinct with-RF waveform, composed at its
 *     first occurrence and cached (dynamic caching) for the later ones, and
 *     with-ADC subsequences without RF are evaluated at every sample directly
 *     from the block-start state by Eq. (4), (5), (6).
 *   All modes give the same result up to floating-point rounding.
 *
 * Units: metres, seconds, tesla, T/m, T*s/m; off-resonance in Hz
 * (B_z gains df / (gamma/2pi)); gamma/2pi = 42.577478518 MHz/T.
 *
 * Memory: "device" pointers are HIP device memory of the context's device
 * (e.g. torch CUDA tensors); "host" pointers are ordinary host memory.
 * Every function returns GBS_OK (0) or a negative status; on failure
 * gbs_last_error(ctx) holds a message.  A context is not thread-safe.
 */
#ifndef GBLOCH_H
#define GBLOCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define GBS_OK 0
#define GBS_E_INVALID (-1) /* bad argument: null pointer, K <= 0, T1/T2 <= 0 or NaN, bad block */
#define GBS_E_STATE (-2)   /* call order: no phantom / sequence, groups missing or stale */
#define GBS_E_HIP (-3)     /* a HIP runtime call or kernel launch failed */
#define GBS_E_NOMEM (-4)   /* device or host allocation failed */
#define GBS_E_WORKSPACE (-5) /* gbs_simulate: workspace null, smaller than gbs_workspace_size, or not 256-byte aligned */

/* ---- block types (Sec. 2.1, Fig. 1) ---------------------------------- */
#define GBS_BLOCK_RF 1    /* with-RF subsequence: stepped, samples not allowed */
#define GBS_BLOCK_ADC 2   /* with-ADC subsequence: stepped, n_samples >= 0 */
#define GBS_BLOCK_RELAX 3 /* relaxation subsequence: closed form over tau with moment */

/* ---- grouping axes (Sec. 2.4) ---------------------------------------- */
#define GBS_AX_X 1u
#define GBS_AX_Y 2u
#define GBS_AX_Z 4u
#define GBS_AX_N 8u   /* no-grads groups: key (T1, T2, dB0) alone */
#define GBS_AX_XZ 16u /* two-axis groups: key (x, z, T1, T2, dB0), for Gx+Gz with-RF subsequences */

/* ---- simulation modes and flags -------------------------------------- */
#define GBS_PLAIN 0
#define GBS_GROUPED 1
#define GBS_CACHED 2
#define GBS_ASYNC 1u      /* enqueue on the context stream and return; no final synchronize */
#define GBS_PROFILE 4u    /* time every sweep launch with HIP events (gbs_stats.pass_kernel_ms) */
#define GBS_SURROGATE 8u  /* GBS_GROUPED, GBS_CACHED: transitions of RF blocks that match the attached surrogate's
                             pulse come from the network, with the spot-check fallback (gbs_set_surrogate) */

/*
 * One subsequence.  RF/ADC blocks cover raster steps
 * [step_offset, step_offset + n_steps) of the waveform arrays; an ADC block's
 * samples are entries [sample_offset, sample_offset + n_samples) of
 * adc_idx (raster boundaries counted from the block start, 0..n_steps,
 * non-decreasing) and of the output signal.  A RELAX block uses tau (s) and
 * moment = int G dt (T*s/m) and ignores the step/sample fields.
 */
typedef struct gbs_block {
    int32_t type;
    int32_t n_samples;
    int64_t step_offset;
    int64_t n_steps;
    int64_t sample_offset;
    double tau;
    double moment[3];
} gbs_block;

typedef struct gbs_info {
    int64_t K;             /* isochromats of the current phantom (0 if none) */
    int64_t n_blocks;      /* blocks of the current sequence */
    int64_t total_steps;   /* raster steps in the waveform arrays */
    int64_t total_samples; /* ADC samples = signal length */
    int64_t stepped_steps; /* raster steps inside RF and ADC blocks */
    int64_t n_groups[3];   /* groups per axis x, y, z; -1 when not built */
    int32_t groups_valid;  /* 1 when groups match the current phantom */
    int32_t device;
    int64_t n_tissue_groups; /* no-grads groups (GBS_AX_N); -1 when not built */
    int64_t n_coils;         /* receive coils of the signal (1 unless gbs_set_coils set more) */
    int64_t n_xz_groups;     /* two-axis (x, z) groups (GBS_AX_XZ); -1 when not built */
} gbs_info;

/* Filled by gbs_simulate when non-null.  Times come from HIP events. */
typedef struct gbs_stats {
    double ms_total;       /* whole simulate call on the device */
    double ms_prepare;     /* grouped: combined transitions and map tables */
    double ms_passes;      /* grouped: streaming passes over all isochromats */
    double ms_adc_eval;    /* grouped: ADC samples from group sums (Eq. 8, 10) */
    double ms_stepped;     /* plain stepping (PLAIN mode, or fallback blocks) */
    int64_t n_passes;      /* grouped operations (group transition and/or group sums) */
    int64_t n_emit_only;   /* operations that only reduce group sums */
    int64_t n_rf_grouped;  /* with-RF blocks applied as group transitions */
    int64_t n_adc_grouped; /* with-ADC blocks evaluated from group sums */
    int64_t n_fallback;    /* RF/ADC blocks stepped per isochromat */
    int64_t n_distinct_rf; /* distinct (waveform, axis) combined transitions composed */
    int64_t n_b1zero;      /* RF-typed blocks with B1 == 0 folded into closed forms */
    double pass_bytes;     /* algorithmic HBM bytes of the sweeps over all isochromats */
    double pass_kernel_ms; /* GBS_PROFILE: sum of the sweep kernel durations */
    int64_t n_sweeps;      /* sweep launches: runs of grouped operations applied in one pass */
    double pass_flops;     /* algorithmic FP32 flops of the sweeps (factor products, maps, transitions, sums) */
    int64_t n_surrogate;   /* GBS_SURROGATE: distinct RF transitions taken from the network */
    int64_t n_surrogate_fallback; /* ... of which failed the spot check and were composed exactly */
    double surrogate_residual;    /* largest spot-check residual max|T_mlp - T_exact| (0 if none) */
    int64_t n_rf_cached;   /* GBS_CACHED: with-RF blocks applied as per-isochromat transitions
                              (n_distinct_rf of them composed, the rest read from the cache) */
    int64_t n_adc_direct;  /* GBS_CACHED: with-ADC blocks evaluated per isochromat and sample */
    double cache_bytes;    /* GBS_CACHED: device bytes of the transition cache (48 per isochromat and entry) */
    double ms_compose;     /* GBS_CACHED + GBS_PROFILE: launches composing and caching transitions */
    double ms_apply;       /* ... launches applying cached transitions or closed-form maps */
    double ms_adc_direct;  /* ... direct ADC launches (with their sample finalize) */
} gbs_stats;

typedef struct gbs_ctx gbs_ctx;

/*
 * Create a context on HIP `device`; work is enqueued on `stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the context.
 * The context also owns one stream of its own at the default priority.  A
 * grouped simulation forks the copy of the final state onto it with an event
 * and makes `stream` wait for it, so work enqueued later on `stream` sees
 * every result.
 * Errors: GBS_E_INVALID (out null, bad device), GBS_E_HIP.
 */
int gbs_create(gbs_ctx **out, int device, void *stream);

/* Release the context and every device buffer it owns.  NULL is a no-op. */
int gbs_destroy(gbs_ctx *ctx);

/*
 * Phantom: K isochromats as device float arrays of length K (Sec. 2.1,
 * Eq. 1): position x, y, z (m), T1, T2 (s, > 0, may be +inf), off-resonance
 * df_hz (Hz) and M0.  The context keeps these pointers (views, no copy) until
 * the next gbs_set_phantom or gbs_destroy; the caller keeps them alive and
 * unchanged.  Validates on the device (NaN, T <= 0 -> GBS_E_INVALID).
 * Invalidates groups.
 */
int gbs_set_phantom(gbs_ctx *ctx, int64_t K, const float *x, const float *y, const float *z,
                    const float *t1, const float *t2, const float *df_hz, const float *m0);

/*
 * Receive coils (Eq. 6 and Eq. 9 with P = n_coils): sens_re, sens_im are
 * device float arrays [n_coils][K] holding S(k, p) of isochromat k (in the
 * phantom's order) for coil p, kept as views until the next gbs_set_coils or
 * gbs_set_phantom (which returns to one coil of unit sensitivity).  Both null
 * with n_coils = 1 selects that default.  With sensitivities the signal of
 * gbs_simulate has n_coils rows in every mode: GBS_GROUPED weights the
 * members of every emission by S before the group sums of each coil (the
 * coil sweep holds each thread's S in registers, read from the context's
 * group-sorted copy), GBS_CACHED weights every directly evaluated term, and
 * per-isochromat stepping (GBS_PLAIN, and stepped readouts in the other
 * modes) adds one weighted sum per coil at every sample, taking at most
 * 256 / n_coils samples per launch.
 * Errors: GBS_E_STATE (no phantom), GBS_E_INVALID (n_coils outside
 * [1, GBS_MAX_COILS], one pointer null, NaN/inf values), GBS_E_HIP.
 */
#define GBS_MAX_COILS 8
int gbs_set_coils(gbs_ctx *ctx, int32_t n_coils, const float *sens_re, const float *sens_im);

/*
 * Sequence (Sec. 2.1, Fig. 1): `blocks` (host, n_blocks entries) over a
 * uniform raster `dt` (s).  Per-step waveforms are host arrays of length
 * total_steps: rf_re, rf_im (B1 in T), gx, gy, gz (T/m); adc_idx is a host
 * int32 array of length total_samples.  Everything is copied; the caller's
 * arrays may be freed after the call.  Validation failures -> GBS_E_INVALID.
 */
int gbs_set_sequence(gbs_ctx *ctx, const gbs_block *blocks, int64_t n_blocks, const float *rf_re,
                     const float *rf_im, const float *gx, const float *gy, const float *gz,
                     int64_t total_steps, const int32_t *adc_idx, int64_t total_samples, double dt);

/*
 * Group the isochromats once (Sec. 2.4, Fig. 2): for each requested axis a
 * (GBS_AX_X | GBS_AX_Y | GBS_AX_Z) the key (r_a, T1, T2, dB0) is compared by
 * exact bit pattern (-0 == +0); equal keys form one group, numbered densely
 * in lexicographic key order.  GBS_AX_N adds the no-grads groups of key
 * (T1, T2, dB0), numbered in ascending (T1, T2, dB0) order: a with-RF
 * subsequence without gradients then composes one transition per such group
 * instead of one per x-group (the result is the same).  GBS_AX_XZ (with
 * GBS_AX_X and GBS_AX_Z) adds the two-axis groups of key (x, z, T1, T2,
 * dB0), which are the runs of equal (x-group, z-group) in the stored copy: a
 * with-RF subsequence whose only gradients are Gx and Gz (an oblique slice)
 * then composes one transition per such group instead of being stepped per
 * isochromat (with-ADC subsequences with two gradients are still stepped).
 * `axes` must include GBS_AX_X (the x groups order the stored copy); blocks
 * whose type needs an axis that was not built are stepped per isochromat,
 * except that no-grads blocks use the x groups when GBS_AX_N is absent.  The
 * context
 * stores a copy of the phantom in group-sorted order (about 12 float/int32
 * words per isochromat).  Synchronizes the stream.
 * Errors: GBS_E_STATE (no phantom), GBS_E_INVALID (no GBS_AX_X, unknown bits,
 * GBS_AX_XZ without GBS_AX_Z),
 * GBS_E_NOMEM, GBS_E_HIP.
 */
int gbs_build_groups(gbs_ctx *ctx, uint32_t axes);

/*
 * Device memory a gbs_simulate call of `mode` needs besides its inputs and
 * outputs, for the current phantom, sequence, groups, coils and surrogate
 * (the largest over the flags of that mode).  The caller allocates it and
 * passes it to gbs_simulate; the library allocates nothing on that path.
 *   GBS_GROUPED: the state in group-sorted order (28 bytes per slot of the
 *     padded layout: three float planes and one (mx, my, mz, 0) row), the
 *     combined-transition and map tables of every grouped subsequence
 *     (Eq. 7, Eq. 4/5), the FP64 group sums of every with-ADC subsequence
 *     (Eq. 9), partial sample sums when blocks are stepped, and the
 *     surrogate's buffers when one is attached (gbs_set_surrogate).
 *   GBS_CACHED: the FP64 state (24 bytes per isochromat), the transition
 *     cache of Sec. 2.2 (48 bytes per isochromat and distinct with-RF
 *     waveform) and partial sample sums.
 *   GBS_PLAIN: partial sample sums, and the FP64 state between launches.
 * Errors: GBS_E_INVALID (bytes null, bad mode), GBS_E_STATE (no phantom or
 * sequence; GBS_GROUPED without groups).
 */
int gbs_workspace_size(gbs_ctx *ctx, int mode, size_t *bytes);

/*
 * Run the sequence on the phantom (Sec. 2.1: Eq. 2-6 per isochromat; the
 * grouped method of Sec. 2.3-2.4, Eq. 7-10; the cached conventional method
 * of Sec. 2.2).  mode = GBS_PLAIN, GBS_GROUPED or GBS_CACHED (GBS_CACHED
 * needs no groups).
 * workspace: device memory of at least gbs_workspace_size(ctx, mode) bytes,
 *          256-byte aligned, owned by the caller.  Its contents are scratch:
 *          nothing is kept in it from one call to the next, and the caller
 *          may reuse it between calls; concurrent calls need separate
 *          workspaces.  Passing the same workspace as the last call avoids
 *          a small upload of the grouped schedule's descriptors.
 * ws_bytes: its size.
 * m_init: device float[3*K] SoA (Mx, My, Mz) or NULL for (0, 0, M0).
 * m_out: device float[3*K] SoA final magnetization (may alias m_init).
 * sig_out: device double[2*n_coils*total_samples], interleaved (re, im), Eq. (6),
 *          coil-major (row p holds coil p; n_coils = 1 without gbs_set_coils).
 * stats: host, nullable.  Without GBS_ASYNC the call synchronizes the stream.
 * GBS_PLAIN steps in FP64 (state and per-step coefficients; in FP32 the
 * rounded coefficients of a constant-gradient readout err the same way at
 * every step, far beyond 1e-5 of M over a long sequence).  GBS_PLAIN and
 * GBS_CACHED keep the state between launches in FP64.
 * GBS_CACHED recomposes its transition cache (3 float4 rows (A_i0, A_i1,
 * A_i2, b_i) of K per distinct with-RF waveform: bit-identical B1 and
 * gradients) in every call.  With-ADC blocks that play RF are stepped per
 * isochromat in every mode.  The schedules this call runs were built by the
 * setters (gbs_set_sequence, gbs_build_groups, gbs_set_coils,
 * gbs_set_surrogate), which also hold their small device arrays.
 * Errors: GBS_E_STATE (no phantom/sequence; GROUPED without valid X groups),
 * GBS_E_INVALID (null outputs, bad mode, unknown flags), GBS_E_WORKSPACE,
 * GBS_E_HIP.
 */
int gbs_simulate(gbs_ctx *ctx, int mode, uint32_t flags, void *workspace, size_t ws_bytes,
                 const float *m_init, float *m_out, double *sig_out, gbs_stats *stats);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * gbs_simulate with the workspace taken from a static device array of
 * GBS_STATIC_WORKSPACE_BYTES that the library holds on every device it runs
 * on until the process ends.  Same arguments, results and errors as
 * gbs_simulate otherwise; calls no allocating routine.  A call whose
 * gbs_workspace_size exceeds the array returns GBS_E_WORKSPACE with the two
 * sizes in gbs_last_error.  Every context on one device shares that device's
 * array, so calls that overlap in time on one device (from different streams
 * or threads) race and must be serialized by the caller; nothing is kept in
 * the array from one call to the next.
 */
#define GBS_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int gbs_simulate_static(gbs_ctx *ctx, int mode, uint32_t flags, const float *m_init, float *m_out,
                        double *sig_out, gbs_stats *stats);

/* Sizes and group counts of the current state. */
int gbs_get_info(gbs_ctx *ctx, gbs_info *info);

/* Last error message of ctx (never NULL); gbs_strerror maps a status code. */
const char *gbs_last_error(const gbs_ctx *ctx);
const char *gbs_strerror(int status);

/*
 * Host-only planning summary (no device needed): classifies the blocks of a
 * sequence (Sec. 2.1, 2.4, 3.1) and counts what GBS_GROUPED would run when
 * groups for `axes` exist.  out[0..7] = grouped RF blocks, grouped ADC
 * blocks, fallback blocks, B1 == 0 RF blocks, streaming passes,
 * emission-only passes, distinct combined transitions, relaxation blocks.
 * Same validation as gbs_set_sequence.
 */
int gbs_plan_summary(const gbs_block *blocks, int64_t n_blocks, const float *rf_re,
                     const float *rf_im, const float *gx, const float *gy, const float *gz,
                     int64_t total_steps, const int32_t *adc_idx, int64_t total_samples, double dt,
                     uint32_t axes, int64_t out[8]);

/*
 * Host-only planning summary of GBS_CACHED (no device needed):
 * out[0..5] = with-RF blocks applied as per-isochromat transitions, distinct
 * transitions composed (cache entries), with-ADC blocks evaluated directly,
 * direct-ADC launches (at most 256 samples each), blocks stepped per
 * isochromat (RF during ADC), RF blocks with B1 == 0 folded into closed forms.
 * Same validation as gbs_set_sequence.
 */
int gbs_plan_cached_summary(const gbs_block *blocks, int64_t n_blocks, const float *rf_re,
                            const float *rf_im, const float *gx, const float *gy, const float *gz,
                            int64_t total_steps, const int32_t *adc_idx, int64_t total_samples,
                            double dt, int64_t out[6]);


/* ==== Pulseq sequence files ============================================
 *
 * Reads the text of a Pulseq sequence file (format version 1.4; other
 * versions -> GBS_E_INVALID) into the block form of gbs_set_sequence
 * (Sec. 2.1, Fig. 1).  Host only, no context and no device.
 *
 * Each Pulseq block of non-zero duration becomes one subsequence: with an
 * ADC event a GBS_BLOCK_ADC block (its RF, if any, stays in it), else with an
 * RF event a GBS_BLOCK_RF block, else a GBS_BLOCK_RELAX block of tau = the
 * block duration and moment = the exact integral of each gradient.  Blocks
 * of zero duration without events (labels) are dropped.  Stepped (RF or ADC)
 * blocks last a whole number of steps of the uniform raster dt (dt <= 0: the
 * file's RF raster time); relaxation blocks keep their exact duration.  In a
 * stepped block every step holds the exact mean over the step of the RF (piecewise
 * constant on the RF raster) and of each gradient (piecewise linear:
 * trapezoids, arbitrary gradients on the default timing with their first and
 * last values, or on a time shape).  ADC sample j lies at
 * delay + (j + 0.5) * dwell from the block start and must fall on a raster
 * boundary.  Units: Hz and Hz/m become T and T/m through gamma/2pi.  The
 * simulated signal ignores the receiver's phase; adc_phase returns it per
 * sample (phase offset + 2 pi * frequency offset * time since the ADC
 * delay, radians) so that a caller can demodulate by exp(-i adc_phase).
 * RF events with a time shape are rejected.  [EXTENSIONS] is ignored.
 * Limits: at most 2^28 stepped raster steps and 2^28 ADC samples per file,
 * 2^26 samples per shape, ids and counts within int32.
 *
 * Two calls.  Query: blocks == NULL; sizes (host int64[3]) receives
 * n_blocks, total_steps, total_samples, nothing else is written.  Fill: the
 * caller passes buffers of at least those sizes in sizes[0..2] and host
 * arrays blocks[n_blocks], rf_re, rf_im, gx, gy, gz [total_steps] (T, T/m),
 * adc_idx[total_samples] (raster boundary from the block start); adc_phase
 * (double[total_samples]) may be NULL; sizes then holds the sizes written.
 * rasters (host double[4], nullable) receives the gradient, RF, ADC and
 * block-duration raster times (s) of the file.  err (host, err_cap bytes,
 * nullable) receives a NUL-terminated message, empty on success.
 * Errors: GBS_E_INVALID (malformed file, unsupported version or event,
 * stepped-block duration or ADC sample off the raster, events outlasting their
 * block, buffers too small or null), GBS_E_NOMEM.
 */
int gbs_pulseq_load(const char *text, int64_t text_len, double dt, int64_t sizes[3],
                    gbs_block *blocks, float *rf_re, float *rf_im, float *gx, float *gy,
                    float *gz, int32_t *adc_idx, double *adc_phase, double rasters[4],
                    char *err, int64_t err_cap);

/* ==== learned RF-transition surrogate ==================================
 *
 * A 5-128-128-128-12 network with SiLU activations that maps the parameters
 * of one isochromat group to the 3x4 combined transition T (Eq. 7) of one
 * fixed with-RF, Gz-only subsequence (the "pulse"): T replaces the exact
 * composition when it passes a spot check.  Inputs per tuple, float[5]:
 *   f_z  = gamma_bar * g_ref * z   (Hz; g_ref = peak |Gz| of the pulse),
 *   f_B0 = dB0 off-resonance (Hz), T1 (s), T2 (s), B1 scale (multiplies B1).
 * Features: f_z, f_B0, ln T1, ln T2, B1 scale, each mapped affinely by
 * (v - center) / scale.  Weights enter the matrix cores as BF16
 * (v_mfma_f32_16x16x32_bf16) with FP32 accumulation and FP32 biases;
 * activations are carried as BF16 hi + lo pairs.  The transition is taken
 * in a frame without the free precession of each half of the pulse,
 * K = P(-a) T P(-a) with P the z rotation of Eq. A2 and
 * a = -2 pi (f_z + f_B0) n_steps dt / 2, and the network outputs
 * Y = 8 (K - K_ref): the residual over a reference transition built from the
 * pulse when it is set.  K_ref takes the pulse's relaxation-free transition
 * at B1 scale 1 (a rotation in this frame, tabulated on 4097 points of
 * f = f_z + f_B0 over +-1600 Hz as angle and axis, interpolated linearly),
 * scales its angle by the B1 scale and splits the relaxation over the pulse
 * around it: A_ref = D R D, b_ref = (1 - E1)(D R e_z + e_z),
 * D = diag(E2, E2, E1), E = exp(-n_steps dt / 2 / T).  T = P(a) (K_ref + Y/8)
 * P(a) is returned.  Training minimises the mean over samples and the 12
 * entries of (Y - 8 (K_exact - K_ref))^2 with Adam on the GPU.
 *
 * Parameter vector (GBS_MLP_PARAMS floats): W1[128][5] b1[128] W2[128][128]
 * b2[128] W3[128][128] b3[128] W4[12][128] b4[12]; layer l computes
 * z = W_l h + b_l.  Transitions are float/double[12] per tuple: A row-major
 * (3x3), then b (M' = A M + b M0).
 */
#define GBS_MLP_PARAMS 35340

typedef struct gbs_mlp gbs_mlp;

typedef struct gbs_train_cfg {
    int32_t epochs;
    int32_t batch;        /* samples per Adam step, multiple of 256 */
    float lr_max, lr_min; /* cosine schedule from lr_max to lr_min over all steps */
    float beta1, beta2, eps;
    uint64_t seed;        /* per-epoch sample order */
} gbs_train_cfg;

/* New network on `device`/`stream` with weights and biases drawn uniformly
 * from +-1/sqrt(fan_in) (seeded); feature normalization defaults to the
 * ranges f_z +-1400 Hz, f_B0 +-100 Hz, T1 0.25-2.5 s, T2 0.03-0.3 s, B1 scale
 * 0.8-1.2.  Errors: GBS_E_INVALID, GBS_E_HIP, GBS_E_NOMEM. */
int gbs_mlp_create(gbs_mlp **out, int device, void *stream, uint64_t seed);
int gbs_mlp_destroy(gbs_mlp *m);
const char *gbs_mlp_last_error(const gbs_mlp *m);

/* The pulse this network models: host waveforms of n_steps raster steps of
 * dt (B1 in T, gradients in T/m).  gx and gy must be zero and gz not all zero
 * (a Gz-only with-RF subsequence, Sec. 2.4).  Copied.  Also builds the
 * reference table from 4097 exact transitions of the pulse (synchronous). */
int gbs_mlp_set_pulse(gbs_mlp *m, const float *rf_re, const float *rf_im, const float *gx,
                      const float *gy, const float *gz, int64_t n_steps, double dt);

/* Feature normalization, host float[5] each (scale != 0). */
int gbs_mlp_set_norm(gbs_mlp *m, const float center[5], const float scale[5]);

/* FP32 master parameters, host float[n], n = GBS_MLP_PARAMS.  set_params
 * also clears the Adam state and step count. */
int gbs_mlp_get_params(gbs_mlp *m, float *params, int64_t n);
int gbs_mlp_set_params(gbs_mlp *m, const float *params, int64_t n);

/* Exact transitions of the pulse (Eq. 7, Eq. A1, A2), FP64: device tuples
 * float[n][5] -> device T double[n][12].  Synchronizes. */
int gbs_mlp_exact(gbs_mlp *m, const float *tuples, int64_t n, double *T);

/* Network transitions: device tuples float[n][5] -> device T float[n][12].
 * Synchronizes. */
int gbs_mlp_infer(gbs_mlp *m, const float *tuples, int64_t n, float *T);

/* Loss and gradient of one batch without an update: n samples (multiple of
 * 64, in order), device T_exact double[n][12]; device grad float[GBS_MLP_PARAMS]
 * in the parameter order above, host *loss.  Synchronizes. */
int gbs_mlp_loss_grad(gbs_mlp *m, const float *tuples, const double *T_exact, int64_t n,
                      float *grad, float *loss);

/* Train with Adam on n samples (n >= cfg->batch): epochs x floor(n / batch)
 * steps, a new seeded sample order every epoch.  loss_hist (host, nullable)
 * receives the batch loss of each step, up to hist_len entries.
 * Synchronizes. */
int gbs_mlp_train(gbs_mlp *m, const float *tuples, const double *T_exact, int64_t n,
                  const gbs_train_cfg *cfg, float *loss_hist, int64_t hist_len);

/* Attach a surrogate to a simulator context (NULL detaches).  Used by
 * gbs_simulate(mode, flags | GBS_SURROGATE) for the with-RF, Gz-only
 * subsequence whose waveform equals the network's pulse bit for bit:
 *   GBS_GROUPED: the network gives T for every z group of the first such
 *     distinct transition; the exact T is composed for n_check seeded
 *     groups (all if fewer);
 *   GBS_CACHED: the network fills the cache entry of the first such
 *     waveform for every isochromat (tuple (f_z, f_B0, T1, T2, 1)) in place
 *     of the per-isochromat FP64 composition (Eq. 7, Sec. 2.2); the exact T
 *     is composed for n_check seeded isochromats.
 * If any checked entry differs by more than tol, the exact transitions of
 * every group or isochromat are used instead (decided on the device, no
 * synchronization).  The network object must outlive its use.  Errors:
 * GBS_E_INVALID (tol <= 0, n_check < 1, device mismatch). */
int gbs_set_surrogate(gbs_ctx *ctx, gbs_mlp *m, float tol, int32_t n_check, uint64_t seed);

/* ==== gradient of the signal (adjoint Bloch simulation) ===================
 *
 * Reverse-mode differentiation of the plain simulation (Eq. 2 with U = D R
 * of Eq. A1, A2 per raster step; Eq. 4, 5 for relaxation blocks; Eq. 6) of
 * the context's phantom and sequence, in FP32 with FP64 sums over
 * isochromats.  The magnetization and the adjoint state are compensated
 * FP32 pairs (hi + lo, each op's increment added by a two-sum), so that the
 * small per-step changes are not rounded away coherently.  Parameters: a
 * complex "parameter pulse" of n_rf samples,
 * played by every listed RF block in place of its own B1, and per-class T1
 * and T2 (isochromat k has class cls[k]; the phantom's own T1/T2 arrays are
 * not used).  For a cotangent w of the signal the backward pass returns the
 * gradient of L = sum_n (w_re[n] Re A_n + w_im[n] Im A_n).
 *
 * The sequence is flattened into ops: a relaxation block, a raster step of
 * a parameter block or with B1 != 0, or a run of raster steps without RF
 * between two sample boundaries (the closed form of Eq. 4, 5 with the run's
 * gradient moment; exact, since all its rotations are about z).  The
 * forward pass stores the state (hi) every `every` ops (3 * K floats per
 * checkpoint, owned by the context); the backward pass steps each segment again from its checkpoint,
 * keeping the state every 8 ops of the segment (3 * K * every / 8 floats,
 * also owned by the context).
 */

/* Forward pass.  cls: device int32[K] in [0, n_classes), n_classes <= 64;
 * t1c, t2c: device float[n_classes] (s, > 0); rf_param: device float[2*n_rf]
 * interleaved (re, im) in T, n_rf <= 3072; param_blocks: host int32 list of
 * RF block indices whose n_steps equals n_rf; every: multiple of 8 in
 * [8, 256].  sig_out: device double[2*total_samples] (re, im).  The context
 * keeps cls, t1c, t2c and rf_param (views) for the backward pass: keep them
 * alive and unchanged until then.  Synchronizes.
 * Errors: GBS_E_STATE (no phantom/sequence), GBS_E_INVALID (limits, block
 * list, class index out of range, T <= 0), GBS_E_NOMEM, GBS_E_HIP. */
int gbs_adj_forward(gbs_ctx *ctx, const int32_t *cls, int32_t n_classes, const float *t1c, const float *t2c,
                    const float *rf_param, int64_t n_rf, const int32_t *param_blocks, int32_t n_param_blocks,
                    int32_t every, double *sig_out);

/* Backward pass of the last gbs_adj_forward: grad_sig device
 * double[2*total_samples] (dL/dRe A_n, dL/dIm A_n); outputs device
 * grad_rf float[2*n_rf] (dL/dRe B1, dL/dIm B1 per sample), grad_t1 and
 * grad_t2 double[n_classes].  May be called repeatedly with different
 * cotangents.  Synchronizes.  Errors: GBS_E_STATE (no forward since the last
 * change of phantom or sequence), GBS_E_INVALID, GBS_E_HIP. */
int gbs_adj_backward(gbs_ctx *ctx, const double *grad_sig, float *grad_rf, double *grad_t1, double *grad_t2);

#ifdef __cplusplus
}
#endif
#endif /* GBLOCH_H */
