// Two-axis groups (key x, z, T1, T2, dB0) for with-RF subsequences whose only
// gradients are Gx and Gz (Sec. 2.4 names such subsequences as the remaining
// case).  In the group-sorted layout every run of equal (x-group, z-group) is
// one such group, so the groups are found from the layout (k_pairs.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace gbs {

// flag[q] = 1 where 4-slot quad q starts a run of equal (gid_x, gid_z), q < n4
hipError_t launch_run_flags(int64_t n4, const int32_t *gid_x, const int32_t *gid_z, uint8_t *flag, hipStream_t st);
// Per run r (first quad first[r]): rtab = (x, T1, T2, dB0 in Hz), rz = z, from the layout arrays
hipError_t launch_run_table(int64_t n_runs, const int32_t *first, const float *xi, const float *zi,
                            const float *t1i, const float *t2i, const float *dfi, float4 *rtab, float *rz,
                            hipStream_t st);
// T = U_{N-1} ... U_0 (Eq. 7, U = D R of Eq. A1, A2) per run in FP64, with
// B_z = Gx x + Gz z + dB0: 12 doubles per run (A row-major, then b)
hipError_t launch_compose_pair(int64_t n_runs, const float4 *rtab, const float *rz, const StepW *wave,
                               int32_t n_steps, double dt, double *out, hipStream_t st);

}  // namespace gbs
