// Learned RF-transition surrogate: a 5-128-128-128-12 SiLU network that maps
// (slice-gradient off-resonance, dB0 off-resonance, T1, T2, B1 scale) to the
// 3x4 affine transition of one RF subsequence (Eq. 7).  Device-side layouts
// shared by k_mlp.hip and api_mlp.cpp.
//
// Parameters (FP32 master copy, flat): W1[128][5] b1[128] W2[128][128] b2[128]
// W3[128][128] b3[128] W4[12][128] b4[12].  Weights enter the matrix cores as
// BF16 (v_mfma_f32_16x16x32_bf16, FP32 accumulation); biases stay FP32.
// Activations are carried as a BF16 pair (hi + lo) so that only the weights
// are rounded to BF16.
//
// Frame: K = P(-a) T P(-a), the transition with the free precession of each
// half of the pulse removed; P(a) is the z rotation of Eq. A2 and
// a = -2 pi (f_z + f_B0) tau/2.  T is recovered exactly as P(a) K P(a)
// (b column: P(a) k_b).
//
// The network predicts the scaled residual kResidualScale (K - K_ref) over a
// reference transition built from the pulse itself: its relaxation-free
// transition at B1 scale 1 in the frame (a rotation), tabulated on
// kRefGrid points of f = f_z + f_B0 over [-kRefFmax, kRefFmax] as rotation
// angle and unit axis (from the unit quaternion, signs continuous along f).
// For a tuple, angle and axis are interpolated linearly in f, the angle is
// scaled by the B1 scale, and the relaxation over the pulse is split around
// the rotation: A_ref = D R D, b_ref = (1 - E1) (D R e_z + e_z),
// D = diag(E2, E2, E1), E = exp(-(tau/2)/T).  The residual is 3-60x smaller
// than K, and so is the error floor that BF16 weights leave on it.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace gbs {

constexpr int kMlpIn = 5, kMlpH = 128, kMlpOut = 12;
constexpr int kOffW1 = 0, kOffB1 = 640, kOffW2 = 768, kOffB2 = 17152, kOffW3 = 17280,
              kOffB3 = 33664, kOffW4 = 33792, kOffB4 = 35328, kMlpParams = 35340;

// Packed MFMA A-operand fragments: 64 lanes x 8 BF16 (1 KiB) each.
// Forward (rows = output neuron, k = input neuron): L1 8 tiles x 1 chunk,
// L2 and L3 8 x 4, L4 1 x 4.  Backward (W^T: rows = input neuron, k = output
// neuron): L2 and L3 8 x 4, L4 8 x 1.
constexpr int kFragFwdL1 = 0, kFragFwdL2 = 8, kFragFwdL3 = 40, kFragFwdL4 = 72, kFragFwd = 76;
constexpr int kFragBwdL2 = 0, kFragBwdL3 = 32, kFragBwdL4 = 64, kFragBwd = 72;

// Weight-gradient tiles (16 x 16, contraction over the batch): L1 8 x 2,
// L2 and L3 8 x 9, L4 1 x 9; the last input tile of each layer is the bias.
constexpr int kGradTiles = 169;

// Training activations, one row per neuron, B samples per row.
constexpr int kActRows = 400;  // H0 (16: 5 inputs + zeros), H1, H2, H3
constexpr int kDzRows = 400;   // dZ1, dZ2, dZ3, dZ4 (16: 12 outputs + zeros)

constexpr int kRefGrid = 4097;          // reference-rotation table points
constexpr double kRefFmax = 1600.0;     // table span of f = f_z + f_B0 [Hz]
constexpr double kResidualScale = 8.0;  // network output = kResidualScale (K - K_ref)

struct MlpNorm {
    float center[5];     // features: f_z [Hz], f_B0 [Hz], ln T1, ln T2, B1 scale
    float inv_scale[5];  // u_k = (feature_k - center_k) * inv_scale_k
    double half;         // tau/2 of the modelled pulse [s]
    const float4 *ref;   // [kRefGrid] (angle, axis x, y, z) of the reference rotation
};

struct MlpTrainArgs {
    const float *tuples;   // [N][5]: f_z, f_B0, T1, T2, B1 scale
    const float *targets;  // [N][12]: K (precession-removed transition)
    int64_t N;
    uint64_t pa, pc;  // sample j of the epoch is (pa * j + pc) mod N
    int64_t j0;       // first sample of this batch within the epoch
    int32_t B;        // batch size (multiple of 64)
    const uint4 *wf, *wb;
    const float *params;
    MlpNorm norm;
    uint16_t *act_h, *act_l, *dz_h, *dz_l;
    float *loss;  // += mean squared error of this batch
};

// Weight gradients of the batch written by k_mlp_train_fb, then Adam.
struct MlpGradAdamArgs {
    const uint16_t *act_h, *act_l, *dz_h, *dz_l;
    int32_t B;  // batch size (multiple of 32)
    float *w, *m, *v;
    uint16_t *wf, *wb;
    float lr, beta1, beta2, eps, corr1, corr2;  // corr = 1 / (1 - beta^t)
    float *grad_out;  // if set: write the gradient and do not update
};

struct MlpInferArgs {
    const float *tuples;  // [.][5], gathered through idx when set
    const int32_t *idx;
    int64_t N;
    const uint4 *wf;
    const float *params;
    MlpNorm norm;
    float *out;  // [N][12] transition T (A row-major, b)
    // Optional tuple source instead of `tuples`: phantom arrays, tuple k =
    // (fz_per_m z[k], df[k], t1[k], t2[k], 1).
    const float *src_z, *src_df, *src_t1, *src_t2;
    double fz_per_m;
    // Optional output instead of `out`: three float4 row planes,
    // rows[i * row_stride + k] = (A_i0, A_i1, A_i2, b_i).
    float4 *rows;
    int64_t row_stride;
};

struct MlpExactArgs {
    const float *tuples;
    const int32_t *idx;  // optional gather
    int64_t N;
    const float4 *wave;  // per step: B1 re, B1 im [T], Gz [T/m], 0
    int32_t n_steps;
    double dt;
    double g_ref;       // f_z = gamma_bar * g_ref * z
    const int32_t *gate;  // optional: run only if *gate != 0
    double *out;        // [N][12]
};

hipError_t launch_mlp_train_fb(const MlpTrainArgs &a, hipStream_t st);
hipError_t launch_mlp_grad_adam(const MlpGradAdamArgs &a, hipStream_t st);
hipError_t launch_mlp_pack(const float *w, uint16_t *wf, uint16_t *wb, hipStream_t st);
hipError_t launch_mlp_infer(const MlpInferArgs &a, hipStream_t st);
hipError_t launch_mlp_exact(const MlpExactArgs &a, hipStream_t st);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t st);
hipError_t launch_mlp_targets(const float *tuples, const double *T, int64_t N, const MlpNorm &norm,
                              float *K, hipStream_t st);
hipError_t launch_surr_tuples(const float4 *gtab, int64_t n, double fz_per_m, float *tuples,
                              hipStream_t st);
hipError_t launch_surr_store(const float *T32, int64_t n, double *T64, hipStream_t st);
hipError_t launch_surr_check(const float *T32, const int32_t *idx, const double *exact, int n_check,
                             float tol, float *residual, int32_t *fallback, hipStream_t st);
hipError_t launch_surr_check_rows(const float4 *rows, int64_t stride, const int32_t *idx, const double *exact,
                                  int n_check, float tol, float *residual, int32_t *fallback, hipStream_t st);
hipError_t launch_surr_iso_tuples(const float *z, const float *df, const float *t1, const float *t2,
                                  const int32_t *idx, int n, double fz_per_m, float *tuples, hipStream_t st);

}  // namespace gbs
