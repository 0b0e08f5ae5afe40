// Host-side state of a surrogate network (gbs_mlp), shared by api_mlp.cpp
// and the simulator's use of it in api.cpp.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mlp.hpp"

struct gbs_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    gbs::MlpNorm norm{};
    // FP32 master parameters, Adam moments, packed BF16 fragments
    float *w = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *wf = nullptr, *wb = nullptr;
    int64_t t = 0;  // Adam steps taken
    // the modelled pulse
    bool has_pulse = false;
    int64_t n_steps = 0;
    double dt = 0.0, g_ref = 0.0;
    std::vector<float> rf_re, rf_im, gz;  // host copy for matching sequence blocks
    float4 *wave = nullptr;               // device: B1 re, B1 im, Gz, 0
    float4 *ref = nullptr;                // device: reference-rotation table (norm.ref)
};

namespace gbs {
// Enqueue MLP transitions for n tuples (device) into T32 (device float[n][12]).
hipError_t mlp_infer_async(const gbs_mlp *m, const float *tuples, const int32_t *idx, int64_t n, float *T32,
                           hipStream_t st);
// Enqueue MLP transitions of phantom isochromats 0 .. n (tuples (g_ref-scaled z,
// df, t1, t2, B1 scale 1)) into three float4 row planes rows[i * stride + k].
hipError_t mlp_infer_rows_async(const gbs_mlp *m, const float *z, const float *df, const float *t1, const float *t2,
                                int64_t n, float4 *rows, int64_t stride, hipStream_t st);
// Enqueue exact transitions (FP64) of the pulse; gate as in MlpExactArgs.
hipError_t mlp_exact_async(const gbs_mlp *m, const float *tuples, const int32_t *idx, int64_t n,
                           const int32_t *gate, double *T64, hipStream_t st);
}  // namespace gbs
