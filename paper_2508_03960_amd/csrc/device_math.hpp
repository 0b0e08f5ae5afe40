// Device helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "consts.hpp"

namespace gbs {

// sin and cos of 2*pi*rev for a phase given in revolutions (cycles).  The
// phase is reduced modulo one turn in FP64, then evaluated by the hardware
// V_SIN_F32 / V_COS_F32, whose input is in revolutions (measured maximum
// absolute error on [-0.5, 0.5]: 1.24e-7).
__device__ __forceinline__ void sincos_rev(double rev, float *s_out, float *c_out) {
    const float r = (float)(rev - rint(rev));
    *s_out = __builtin_amdgcn_sinf(r);
    *c_out = __builtin_amdgcn_cosf(r);
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

}  // namespace gbs
