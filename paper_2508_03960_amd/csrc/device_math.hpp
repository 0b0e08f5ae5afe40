// Device helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "consts.hpp"

namespace gbs {

// sin and cos of 2*pi*rev for a phase given in revolutions (cycles).  The
// phase is reduced in FP64 to the nearest quarter turn, the remainder
// |t| <= pi/4 is evaluated in FP32 with the Taylor series of sin (to t^9)
// and cos (to t^10), whose truncation errors are below 2e-9 on that range.
__device__ __forceinline__ void sincos_rev(double rev, float *s_out, float *c_out) {
    const double q4 = 4.0 * (rev - rint(rev));  // quarter turns in [-2, 2]
    const double q = rint(q4);
    const float t = (float)((q4 - q) * 1.5707963267948966192313216916398);
    const float t2 = t * t;
    float sp = fmaf(t2, 2.7557319223985891e-6f, -1.9841269841269841e-4f);
    sp = fmaf(t2, sp, 8.3333333333333333e-3f);
    sp = fmaf(t2, sp, -1.6666666666666667e-1f);
    sp = fmaf(t2 * t, sp, t);
    float cp = fmaf(t2, -2.7557319223985891e-7f, 2.4801587301587302e-5f);
    cp = fmaf(t2, cp, -1.3888888888888889e-3f);
    cp = fmaf(t2, cp, 4.1666666666666667e-2f);
    cp = fmaf(t2, cp, -0.5f);
    cp = fmaf(t2, cp, 1.0f);
    const int k = ((int)q) & 3;  // rotate (sin t, cos t) by k quarter turns
    float s = sp, c = cp;
    if (k == 1) { s = cp; c = -sp; }
    else if (k == 2) { s = -sp; c = -cp; }
    else if (k == 3) { s = -cp; c = sp; }
    *s_out = s;
    *c_out = c;
}

// ---- wavefront (64-lane) sums through DPP; the total lands in lane 63 ----
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ float wave_sum_lane63(float v) {
    v += dpp_f32<0xb1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f32<0x4e>(v);   // quad_perm [2,3,0,1]
    v += dpp_f32<0x114>(v);  // row_shr:4
    v += dpp_f32<0x118>(v);  // row_shr:8  -> lane 15 of each row holds the row sum
    v += dpp_f32<0x142>(v);  // row_bcast:15
    v += dpp_f32<0x143>(v);  // row_bcast:31 -> lane 63 holds the wave sum
    return v;
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_lane63_f64(double v) {
    v += dpp_f64<0xb1>(v);
    v += dpp_f64<0x4e>(v);
    v += dpp_f64<0x114>(v);
    v += dpp_f64<0x118>(v);
    v += dpp_f64<0x142>(v);
    v += dpp_f64<0x143>(v);
    return v;
}

// Compensated (Kahan) accumulation of x into (sum, comp).
__device__ __forceinline__ void kahan_add(float &sum, float &comp, float x) {
    const float y = x - comp;
    const float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

}  // namespace gbs
