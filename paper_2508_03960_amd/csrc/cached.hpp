// The conventional accelerated method (Sec. 2.2) that the grouped update is
// compared with: per-isochromat combined transitions T_k (Eq. 7), composed at
// the first occurrence of a with-RF waveform and cached (dynamic caching), and
// with-ADC subsequences evaluated per isochromat and sample from the state at
// the block start (Eq. 4, 5, 6).  Argument blocks and launchers of
// k_cached.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace gbs {

// One operation on every isochromat: the pending closed-form map (Eq. 4, 5),
// then, by launch mode,
//   kCacheMap:     nothing more;
//   kCacheApply:   M <- A M + b M0 with the cached entry (3 float4 rows per
//                  isochromat: (A_i0, A_i1, A_i2, b_i));
//   kCacheCompose: compose T = U_{N-1} ... U_0 (U = D R, Eq. A1, A2) over the
//                  block's raster steps in FP64, store it as the entry, apply it.
enum { kCacheMap = 0, kCacheApply = 1, kCacheCompose = 2 };

struct CachedArgs {
    int64_t K;
    PhantomPtrs ph;
    // state in: FP64 SoA [3][K] when s64_in is set, else FP32 min_* when set,
    // else (0, 0, M0)
    const double *s64_in;
    const float *min_x, *min_y, *min_z;
    // state out: FP64 SoA [3][K] when s64_out is set, else FP32 mout_*
    double *s64_out;
    float *mout_x, *mout_y, *mout_z;
    int32_t has_pre;
    double pre_tau;
    double pre_cyc[3];  // gamma_bar * moment (cycles per metre)
    float4 *cache;      // rows [3][K] of the entry (apply, compose)
    const StepW *wave;  // compose: first raster step of the block
    int32_t n_steps;    // compose
    double dt;
    double gdt;  // gamma * dt (rad / T)
    // optional: the launch does nothing unless *gate == gate_value (a device
    // flag set by an earlier kernel on the stream, e.g. a surrogate's spot check)
    const int32_t *gate;
    int32_t gate_value;
};

// Samples of one with-ADC block without RF.  Sample n sees the block-start
// state M after the map with phase c_n . r + tau_n * df (cycles) and T2 decay
// over tau_n; samp[n] = (c_n (cycles per metre, 3 components), tau_n (s)),
// each including the maps pending before the block.
struct DirectAdcArgs {
    int64_t K;
    PhantomPtrs ph;
    const double *s64_in;         // as CachedArgs
    const float *min_x, *min_y;
    const double4 *samp;
    int32_t n_samples;  // 1 .. 256
    // Receive coils (Eq. 6 with S(k, p)): sensitivities [n_coils][K] in the
    // caller's order, or null for one coil of unit sensitivity
    const float *coil_re, *coil_im;
    int32_t n_coils;     // 1 .. kMaxCoils
    double2 *partial;    // [n_coils][gridDim.x][n_samples] per-workgroup sums
};

constexpr int kMaxCoils = 8;

hipError_t launch_cached(const CachedArgs &a, int mode, hipStream_t st);
int direct_adc_grid(int64_t K);
hipError_t launch_direct_adc(const DirectAdcArgs &a, int grid, hipStream_t st);

}  // namespace gbs
