// Device grouping helpers (k_groups.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gbs {

size_t group_scratch_bytes(int64_t K);
hipError_t group_axis(int64_t K, const float *coord, const float *t1, const float *t2, const float *df,
                      void *scratch, size_t scratch_bytes, int32_t *gid_nat, float4 *gtab,
                      int32_t *gcount, int32_t *order, int64_t *n_groups, hipStream_t st);
hipError_t build_layout(int64_t K, const int32_t *gid_x, const int32_t *gid_z, void *scratch, size_t scratch_bytes,
                        int32_t *perm, int32_t *src, int64_t Kpad_cap, int64_t *kint, hipStream_t st);
hipError_t launch_invert(int64_t n, const int32_t *perm, int32_t *inv, hipStream_t st);
hipError_t launch_zero_padding(int64_t n, const int32_t *perm, float *m0, hipStream_t st);
hipError_t launch_gather_f32(int64_t K, int64_t Kpad, const int32_t *perm, const float *src, float *dst,
                             hipStream_t st);
// dst[i] <- src[perm[i]], 0 where perm[i] < 0 (layout padding), for i < n
hipError_t launch_gather_padded(int64_t n, const int32_t *perm, const float *src, float *dst, hipStream_t st);
// *bad <- 1 if any of a[0 .. n) is NaN or infinite (*bad is not cleared)
hipError_t launch_check_finite(int64_t n, const float *a, int *bad, hipStream_t st);
// dst row g (12 doubles) <- src row map[g], for g < n
hipError_t launch_expand_rows(const double *src, const int32_t *map, int64_t n, double *dst, hipStream_t st);
hipError_t launch_gather_i32(int64_t K, int64_t Kpad, const int32_t *perm, const int32_t *src,
                             int32_t *dst, hipStream_t st);

}  // namespace gbs
