// Receive coils for the per-isochromat stepping kernel (Eq. 6 with S(k, p)):
// the sensitivities of the launch's isochromats, in the launch's order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace gbs {

constexpr int kPlainMaxCoils = 8;

struct PlainCoils {
    const float *re, *im;  // coil p of isochromat k: re[p * stride + k], im[p * stride + k]
    int64_t stride;
    int32_t n;  // 1 .. kPlainMaxCoils
};

// k_plain with coil sums: every sample of the launch gets one sum per coil,
// written as partials [coil][grid][n_samples]; needs n_samples * n <= 256.
hipError_t launch_plain_coils(const PlainArgs &a, const PlainCoils &c, bool has_b1, int grid, hipStream_t st);

}  // namespace gbs
