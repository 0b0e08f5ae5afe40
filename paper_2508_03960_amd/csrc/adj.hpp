// Adjoint (reverse-mode) Bloch simulation: device-side layouts shared by
// k_adjoint.hip and api_adj.cpp.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace gbs {

constexpr int kAdjWG = 256;          // isochromats per workgroup (one per thread)
constexpr int kAdjSub = 8;           // ops per recomputed sub-segment (states in registers)
constexpr int kAdjMaxEvery = 256;    // largest checkpoint interval
constexpr int kAdjMaxClasses = 64;
constexpr int kAdjMaxRf = 3072;      // parameter-pulse samples (gradient accumulated in LDS, 24 KiB)

// One op of the flattened sequence: a raster step (Eq. A1, A2) or a
// relaxation block (Eq. 4, 5).  64 bytes.
struct AdjOp {
    float b1r, b1i, gx, gy, gz;  // raster: B1 [T] (unless param >= 0) and gradients [T/m]
    int32_t param;               // raster: sample of the parameter pulse, or -1
    int32_t kind;                // 0 raster step, 1 relaxation block
    int32_t pad;
    double tau;                  // relaxation: duration [s]
    double cyc[3];               // relaxation: gamma_bar * gradient moment [cycles/m]
};

struct AdjArgs {
    int64_t K;
    const float *x, *y, *z, *df, *m0;
    const int32_t *cls;
    const float *t1c, *t2c;
    int32_t n_classes;
    const AdjOp *ops;
    int32_t n_ops;
    const float2 *rfp;  // parameter pulse, n_rf samples
    int32_t n_rf;
    const int32_t *sstart;  // [n_ops + 2]: samples taken at boundary p are sid[sstart[p] .. sstart[p+1])
    const int32_t *sid;
    double dt;
    int32_t every;       // checkpoint interval in ops (multiple of kAdjSub, <= kAdjMaxEvery)
    float *ckpt;         // [n_ckpt][3][K]: state at boundaries 0, every, 2 every, ...
    float *sub;          // backward: [every / kAdjSub][3][K] sub-checkpoints of the current segment
    int32_t N;           // samples
    double2 *sig_part;   // forward: [grid][N] per-workgroup sums
    const double2 *w;    // backward: cotangent of the signal, [N] (d/dRe, d/dIm)
    float2 *grf_part;    // backward: [grid][n_rf]
    double2 *gt_part;    // backward: [grid][n_classes] (dL/dT1, dL/dT2)
};

hipError_t launch_adj_forward(const AdjArgs &a, hipStream_t st);
hipError_t launch_adj_backward(const AdjArgs &a, hipStream_t st);
hipError_t launch_adj_validate(int64_t K, const int32_t *cls, int n_classes, const float *t1c, const float *t2c,
                               int *flag, hipStream_t st);
hipError_t launch_adj_finalize(const AdjArgs &a, double *sig, float *grad_rf, double *grad_t1, double *grad_t2,
                               bool forward, hipStream_t st);

}  // namespace gbs
