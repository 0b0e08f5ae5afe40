// Grouping of isochromats (Sec. 2.4, Fig. 2) on the device.
//
// For an axis a the key of isochromat k is (r_a, T1, T2, dB0), compared by
// exact bit pattern with -0 folded onto +0.  Keys are made order-preserving
// 32-bit words, packed as two 64-bit halves and sorted with two stable LSD
// radix passes (low half, then high half), carrying the isochromat index.
// Equal neighbours share a group id; ids are dense in lexicographic key order.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "groups.hpp"
#include "kernels.hpp"

namespace gbs {

// rocPRIM device primitives on int32 counts (stable LSD radix sort of 64-bit
// keys with an int32 payload; inclusive and exclusive sums).  With tmp null
// they report the temporary bytes they need in *bytes.
static hipError_t sort_pairs(void *tmp, size_t *bytes, const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                             int32_t *vout, int64_t n, hipStream_t st) {
    return rocprim::radix_sort_pairs(tmp, *bytes, kin, kout, vin, vout, (unsigned int)n, 0u, 64u, st);
}
static hipError_t inclusive_sum(void *tmp, size_t *bytes, const int32_t *in, int32_t *out, int64_t n, hipStream_t st) {
    return rocprim::inclusive_scan(tmp, *bytes, in, out, (size_t)n, rocprim::plus<int32_t>(), st);
}
static hipError_t exclusive_sum(void *tmp, size_t *bytes, const int32_t *in, int32_t *out, int64_t n, hipStream_t st) {
    return rocprim::exclusive_scan(tmp, *bytes, in, out, (int32_t)0, (size_t)n, rocprim::plus<int32_t>(), st);
}

__device__ __forceinline__ uint32_t ordered_bits(float f) {
    const uint32_t u = __float_as_uint(f + 0.0f);  // -0 -> +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ void k_keys(int64_t K, const float *__restrict__ c, const float *__restrict__ t1,
                       const float *__restrict__ t2, const float *__restrict__ df, uint64_t *hi,
                       uint64_t *lo, int32_t *idx) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x) {
        hi[i] = ((uint64_t)ordered_bits(c[i]) << 32) | ordered_bits(t1[i]);
        lo[i] = ((uint64_t)ordered_bits(t2[i]) << 32) | ordered_bits(df[i]);
        idx[i] = (int32_t)i;
    }
}

__global__ void k_gather_u64(int64_t K, const uint64_t *__restrict__ src, const int32_t *__restrict__ idx,
                             uint64_t *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[idx[i]];
}

__global__ void k_heads(int64_t K, const uint64_t *__restrict__ hi, const uint64_t *__restrict__ lo,
                        int32_t *__restrict__ flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = (i == 0 || hi[i] != hi[i - 1] || lo[i] != lo[i - 1]) ? 1 : 0;
}

// ids = inclusive scan of the head flags (1-based).
__global__ void k_assign(int64_t K, const int32_t *__restrict__ ids, const int32_t *__restrict__ order,
                         const float *__restrict__ c, const float *__restrict__ t1,
                         const float *__restrict__ t2, const float *__restrict__ df,
                         int32_t *__restrict__ gid_nat, float4 *__restrict__ gtab,
                         int32_t *__restrict__ gstart) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t g = ids[i] - 1;
        const int32_t k = order[i];
        gid_nat[k] = g;
        if (i == 0 || ids[i - 1] != ids[i]) {
            gtab[g] = make_float4(c[k], t1[k], t2[k], df[k]);
            gstart[g] = (int32_t)i;
        }
    }
}

__global__ void k_counts(int64_t G, int64_t K, const int32_t *__restrict__ gstart, int32_t *__restrict__ gcount) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x)
        gcount[g] = (int32_t)((g + 1 < G ? gstart[g + 1] : K) - gstart[g]);
}

__global__ void k_gather_f32(int64_t K, int64_t Kpad, const int32_t *__restrict__ perm,
                             const float *__restrict__ src, float *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Kpad; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = i < K ? src[perm[i]] : 0.0f;
}

__global__ void k_gather_i32(int64_t K, int64_t Kpad, const int32_t *__restrict__ perm,
                             const int32_t *__restrict__ src, int32_t *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Kpad; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = i < K ? src[perm[i]] : 0;
}

__global__ void k_validate(int64_t K, PhantomPtrs ph, int *bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x) {
        const float t1 = ph.t1[i], t2 = ph.t2[i];
        const bool ok = (t1 > 0.f) && (t2 > 0.f) && isfinite(ph.x[i]) && isfinite(ph.y[i]) &&
                        isfinite(ph.z[i]) && isfinite(ph.df[i]) && isfinite(ph.m0[i]);
        if (!ok) atomicOr(bad, 1);
    }
}

// ---- padded group-sorted layout ---------------------------------------------
// Isochromats are ordered by (x-group, z-group, index) and every run of equal
// (x-group, z-group) is padded to a multiple of 8 with copies of its first
// member carrying M0 = 0.  A thread's 8 (or 4) consecutive isochromats then always
// share both groups.
__global__ void k_pair_keys(int64_t K, const int32_t *__restrict__ gx, const int32_t *__restrict__ gz,
                            uint64_t *__restrict__ key, int32_t *__restrict__ idx) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x) {
        key[i] = ((uint64_t)(uint32_t)gx[i] << 32) | (gz ? (uint32_t)gz[i] : 0u);
        idx[i] = (int32_t)i;
    }
}

__global__ void k_key_heads(int64_t K, const uint64_t *__restrict__ key, int32_t *__restrict__ flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

__global__ void k_run_start(int64_t K, const int32_t *__restrict__ rid, int32_t *__restrict__ rstart) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x)
        if (i == 0 || rid[i] != rid[i - 1]) rstart[rid[i] - 1] = (int32_t)i;
}

__global__ void k_run_plen(int64_t R, int64_t K, const int32_t *__restrict__ rstart, int32_t *__restrict__ plen) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t L = (int32_t)((r + 1 < R ? rstart[r + 1] : K) - rstart[r]);
        plen[r] = (L + 7) & ~7;  // 8-isochromat sweep threads never straddle a run
    }
}

__global__ void k_place(int64_t K, const int32_t *__restrict__ rid, const int32_t *__restrict__ rstart,
                        const int32_t *__restrict__ pstart, const int32_t *__restrict__ order,
                        int32_t *__restrict__ perm, int32_t *__restrict__ src) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = rid[i] - 1;
        const int64_t pos = (int64_t)pstart[r] + (i - rstart[r]);
        perm[pos] = order[i];
        src[pos] = order[i];
    }
}

__global__ void k_pad(int64_t R, int64_t K, const int32_t *__restrict__ rstart, const int32_t *__restrict__ pstart,
                      const int32_t *__restrict__ plen, const int32_t *__restrict__ order, int32_t *__restrict__ perm,
                      int32_t *__restrict__ src) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t L = (int32_t)((r + 1 < R ? rstart[r + 1] : K) - rstart[r]);
        const int32_t first = order[rstart[r]];
        for (int32_t j = L; j < plen[r]; ++j) {
            perm[pstart[r] + j] = -1;
            src[pstart[r] + j] = first;
        }
    }
}

__global__ void k_fill_tail(int64_t from, int64_t to, int32_t *__restrict__ perm, int32_t *__restrict__ src) {
    for (int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < to; i += (int64_t)gridDim.x * blockDim.x) {
        perm[i] = -1;
        src[i] = 0;
    }
}

__global__ void k_zero_padding(int64_t n, const int32_t *__restrict__ perm, float *__restrict__ m0) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (perm[i] < 0) m0[i] = 0.0f;
}

static dim3 grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return dim3((unsigned)g);
}

hipError_t launch_validate_phantom(int64_t K, const PhantomPtrs &ph, int *bad, hipStream_t st) {
    hipLaunchKernelGGL(k_validate, grid_for(K), dim3(256), 0, st, K, ph, bad);
    return hipGetLastError();
}

hipError_t launch_gather_f32(int64_t K, int64_t Kpad, const int32_t *perm, const float *src, float *dst,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_gather_f32, grid_for(Kpad), dim3(256), 0, st, K, Kpad, perm, src, dst);
    return hipGetLastError();
}

hipError_t launch_gather_i32(int64_t K, int64_t Kpad, const int32_t *perm, const int32_t *src,
                             int32_t *dst, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_i32, grid_for(Kpad), dim3(256), 0, st, K, Kpad, perm, src, dst);
    return hipGetLastError();
}

__global__ void k_gather_padded(int64_t n, const int32_t *__restrict__ perm, const float *__restrict__ src,
                                float *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = perm[i];
        dst[i] = k >= 0 ? src[k] : 0.0f;
    }
}

__global__ void k_check_finite(int64_t n, const float *__restrict__ a, int *__restrict__ bad) {
    bool ok = true;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        ok = ok && isfinite(a[i]);
    if (!ok) *bad = 1;
}

__global__ void k_expand_rows(const double *__restrict__ src, const int32_t *__restrict__ map, int64_t n,
                              double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= 12 * n) return;
    const int64_t g = i / 12;
    dst[i] = src[12 * (int64_t)map[g] + (i - 12 * g)];
}

hipError_t launch_gather_padded(int64_t n, const int32_t *perm, const float *src, float *dst, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_padded, grid_for(n), dim3(256), 0, st, n, perm, src, dst);
    return hipGetLastError();
}

hipError_t launch_check_finite(int64_t n, const float *a, int *bad, hipStream_t st) {
    hipLaunchKernelGGL(k_check_finite, grid_for(n), dim3(256), 0, st, n, a, bad);
    return hipGetLastError();
}

hipError_t launch_expand_rows(const double *src, const int32_t *map, int64_t n, double *dst, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_expand_rows, dim3((unsigned)((12 * n + 255) / 256)), dim3(256), 0, st, src, map, n, dst);
    return hipGetLastError();
}

// Build the padded layout from natural-order x (and optional z) group ids.
// perm[pos] = isochromat at internal position pos or -1 (padding); src[pos] =
// the isochromat whose parameters the position copies.  perm/src need room
// for Kpad_cap entries; *kint receives the padded count (a multiple of 8).
hipError_t build_layout(int64_t K, const int32_t *gid_x, const int32_t *gid_z, void *scratch, size_t scratch_bytes,
                        int32_t *perm, int32_t *src, int64_t Kpad_cap, int64_t *kint, hipStream_t st) {
    char *p = (char *)scratch;
    auto take = [&](size_t n) {
        char *r = p;
        p += (n + 255) & ~(size_t)255;
        return (void *)r;
    };
    uint64_t *key = (uint64_t *)take(8 * K), *key2 = (uint64_t *)take(8 * K);
    int32_t *idx = (int32_t *)take(4 * K), *order = (int32_t *)take(4 * K), *flag = (int32_t *)take(4 * K);
    int32_t *rid = (int32_t *)take(4 * K), *rstart = (int32_t *)take(4 * K), *plen = (int32_t *)take(4 * K);
    int32_t *pstart = (int32_t *)take(4 * K);
    const size_t used = (size_t)(p - (char *)scratch);
    if (used > scratch_bytes) return hipErrorInvalidValue;
    void *tmp = p;
    size_t tmp_bytes = scratch_bytes - used;
    const dim3 g = grid_for(K);
    hipError_t e;
    hipLaunchKernelGGL(k_pair_keys, g, dim3(256), 0, st, K, gid_x, gid_z, key, idx);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = sort_pairs(tmp, &tmp_bytes, key, key2, idx, order, K, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_key_heads, g, dim3(256), 0, st, K, key2, flag);
    if ((e = inclusive_sum(tmp, &tmp_bytes, flag, rid, K, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_run_start, g, dim3(256), 0, st, K, rid, rstart);
    int32_t R = 0;
    if ((e = hipMemcpyAsync(&R, rid + (K - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_run_plen, grid_for(R), dim3(256), 0, st, (int64_t)R, K, rstart, plen);
    if ((e = exclusive_sum(tmp, &tmp_bytes, plen, pstart, R, st)) != hipSuccess) return e;
    int32_t last[2] = {0, 0};
    if ((e = hipMemcpyAsync(&last[0], pstart + (R - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(&last[1], plen + (R - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    const int64_t n = (int64_t)last[0] + last[1];
    if (n > Kpad_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_place, g, dim3(256), 0, st, K, rid, rstart, pstart, order, perm, src);
    hipLaunchKernelGGL(k_pad, grid_for(R), dim3(256), 0, st, (int64_t)R, K, rstart, pstart, plen, order, perm, src);
    if (Kpad_cap > n) hipLaunchKernelGGL(k_fill_tail, grid_for(Kpad_cap - n), dim3(256), 0, st, n, Kpad_cap, perm, src);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    *kint = n;
    return hipSuccess;
}

__global__ void k_invert(int64_t n, const int32_t *__restrict__ perm, int32_t *__restrict__ inv) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (perm[i] >= 0) inv[perm[i]] = (int32_t)i;
}

hipError_t launch_invert(int64_t n, const int32_t *perm, int32_t *inv, hipStream_t st) {
    hipLaunchKernelGGL(k_invert, grid_for(n), dim3(256), 0, st, n, perm, inv);
    return hipGetLastError();
}

hipError_t launch_zero_padding(int64_t n, const int32_t *perm, float *m0, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_padding, grid_for(n), dim3(256), 0, st, n, perm, m0);
    return hipGetLastError();
}

size_t group_scratch_bytes(int64_t K) {
    size_t sort_tmp = 0, scan_tmp = 0, escan_tmp = 0;
    const bool sized = sort_pairs(nullptr, &sort_tmp, nullptr, nullptr, nullptr, nullptr, K, 0) == hipSuccess &&
                       inclusive_sum(nullptr, &scan_tmp, nullptr, nullptr, K, 0) == hipSuccess &&
                       exclusive_sum(nullptr, &escan_tmp, nullptr, nullptr, K, 0) == hipSuccess;
    size_t tmp = sort_tmp > scan_tmp ? sort_tmp : scan_tmp;
    if (escan_tmp > tmp) tmp = escan_tmp;
    // a failed size query leaves generous room; the sorts and scans report their own errors
    if (!sized) tmp = ((size_t)64 << 20) + 16 * (size_t)K;
    // the larger of group_axis (4 u64 + 3 i32 arrays) and build_layout (2 u64 + 7 i32), plus tmp
    return 4 * sizeof(uint64_t) * K + 7 * sizeof(int32_t) * K + tmp + 16 * 256;
}

// Group one axis.  coord = r_a of every isochromat (natural order).  Writes
// gid_nat[K] (natural order), gtab[n_groups] = (coord, T1, T2, df) and
// gcount[n_groups] (gtab and gcount need room for K entries), order[K] =
// isochromat indices sorted by key (stable), and returns the group count
// through *n_groups (synchronizes the stream).
hipError_t group_axis(int64_t K, const float *coord, const float *t1, const float *t2, const float *df,
                      void *scratch, size_t scratch_bytes, int32_t *gid_nat, float4 *gtab,
                      int32_t *gcount, int32_t *order, int64_t *n_groups, hipStream_t st) {
    char *p = (char *)scratch;
    auto take = [&](size_t n) {
        char *r = p;
        p += (n + 255) & ~(size_t)255;
        return (void *)r;
    };
    uint64_t *hi = (uint64_t *)take(8 * K), *lo = (uint64_t *)take(8 * K);
    uint64_t *k2 = (uint64_t *)take(8 * K), *k3 = (uint64_t *)take(8 * K);
    int32_t *idx0 = (int32_t *)take(4 * K), *idx1 = (int32_t *)take(4 * K), *flag = (int32_t *)take(4 * K);
    const size_t used = (size_t)(p - (char *)scratch);
    if (used > scratch_bytes) return hipErrorInvalidValue;
    void *tmp = p;
    size_t tmp_bytes = scratch_bytes - used;
    const dim3 g = grid_for(K);
    hipError_t e;
    hipLaunchKernelGGL(k_keys, g, dim3(256), 0, st, K, coord, t1, t2, df, hi, lo, idx0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // LSD: low half first (carry indices), then the high half of the same records.
    if ((e = sort_pairs(tmp, &tmp_bytes, lo, k2, idx0, idx1, K, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_u64, g, dim3(256), 0, st, K, hi, idx1, k3);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = sort_pairs(tmp, &tmp_bytes, k3, hi, idx1, order, K, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_u64, g, dim3(256), 0, st, K, lo, order, k2);  // low half in final order
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_heads, g, dim3(256), 0, st, K, hi, k2, flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = inclusive_sum(tmp, &tmp_bytes, flag, idx0, K, st)) != hipSuccess) return e;
    int32_t *gstart = idx1;  // the first sort's payload is no longer needed
    hipLaunchKernelGGL(k_assign, g, dim3(256), 0, st, K, idx0, order, coord, t1, t2, df, gid_nat, gtab, gstart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int32_t last = 0;
    if ((e = hipMemcpyAsync(&last, idx0 + (K - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_counts, grid_for(last), dim3(256), 0, st, (int64_t)last, K, gstart, gcount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    *n_groups = last;
    return hipSuccess;
}

}  // namespace gbs
