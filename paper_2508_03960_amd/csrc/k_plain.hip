// Plain per-isochromat stepping on gfx950 (the conventional method that the
// grouped update is measured against, Sec. 2.2).
//
// One thread carries kIso isochromats in registers through every raster step
// of a block: U = D R (Eq. 2, Eq. A1, Eq. A2).  The waveform value of a step
// is the same for every lane, so it is one scalar load per step.
//
// FP32 is used in increment form so that rounding does not bias the state:
//   R M = M + a (B x M) + b (B (B . M) - |B|^2 M),
//   a = sin(theta)/|B|,  b = (1 - cos theta)/|B|^2,  theta = -gamma |B| dt,
// with a, b from their power series in q = theta^2 (no sqrt, no division, and
// R = I falls out at B = 0); relaxation as M -= (1 - E) M with
// 1 - E = -expm1(-dt/T) computed once per isochromat.
//
// ADC samples (Eq. 6): at each sample boundary a wavefront sums its lanes with
// DPP, lane 63 adds the wave total into a per-wave compensated (Kahan) FP32
// accumulator in LDS; at the end each workgroup writes one FP64 partial per
// sample, and a finalize kernel adds the partials in a fixed order.
#include "device_math.hpp"
#include "kernels.hpp"

namespace gbs {

constexpr int kPlainBlock = 256;
constexpr int kIso = 2;
constexpr int kTile = kPlainBlock * kIso;
constexpr float kQMax = 1.0f;  // series used while theta^2 <= 1

// a = sin(theta)/|B| = -gdt * S(q), b = (1 - cos theta)/|B|^2 = gdt^2 * C(q),
// S(q) = sum (-q)^n / (2n+1)!, C(q) = sum (-q)^n / (2n+2)!, n = 0..5.
__device__ __forceinline__ void rot_coeffs(float B2, float gdt, float k2, float &a, float &b) {
    const float q = k2 * B2;
    if (q <= kQMax) {
        float S = fmaf(q, -2.5052108385441719e-8f, 2.7557319223985891e-6f);
        S = fmaf(q, S, -1.9841269841269841e-4f);
        S = fmaf(q, S, 8.3333333333333333e-3f);
        S = fmaf(q, S, -1.6666666666666667e-1f);
        S = fmaf(q, S, 1.0f);
        float C = fmaf(q, -2.0876756987868099e-9f, 2.7557319223985891e-7f);
        C = fmaf(q, C, -2.4801587301587302e-5f);
        C = fmaf(q, C, 1.3888888888888889e-3f);
        C = fmaf(q, C, -4.1666666666666667e-2f);
        C = fmaf(q, C, 0.5f);
        a = -gdt * S;
        b = k2 * C;
    } else {
        const float nb = sqrtf(B2);
        float sh, ch;
        sincosf(0.5f * gdt * nb, &sh, &ch);
        a = -2.0f * sh * ch / nb;
        b = 2.0f * sh * sh / B2;
    }
}

template <bool HAS_B1>
__global__ __launch_bounds__(kPlainBlock) void k_plain(PlainArgs a) {
    extern __shared__ float4 acc[];  // [4 waves][n_samples]: (sum re, comp re, sum im, comp im)
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int ns = a.n_samples;
    for (int i = tid; i < 4 * ns; i += kPlainBlock) acc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    const float gdt = a.gdt;
    const float k2 = gdt * gdt;
    const StepW *__restrict__ wave_ptr = a.wave;
    const int32_t *__restrict__ sidx = a.sidx;

    for (int64_t base = (int64_t)blockIdx.x * kTile; base < a.K; base += (int64_t)gridDim.x * kTile) {
        float X[kIso], Y[kIso], Z[kIso], boff[kIso], e1m[kIso], e2m[kIso], M0[kIso];
        float mx[kIso], my[kIso], mz[kIso];
#pragma unroll
        for (int i = 0; i < kIso; ++i) {
            const int64_t k = base + (int64_t)i * kPlainBlock + tid;
            if (k < a.K) {
                X[i] = a.ph.x[k];
                Y[i] = a.ph.y[k];
                Z[i] = a.ph.z[k];
                const double t1 = a.ph.t1[k], t2 = a.ph.t2[k], df = a.ph.df[k];
                M0[i] = a.ph.m0[k];
                boff[i] = (float)(df / kGammaBar);
                e1m[i] = (float)(-expm1(-a.dt / t1));
                e2m[i] = (float)(-expm1(-a.dt / t2));
                if (a.min_x) {
                    mx[i] = a.min_x[k];
                    my[i] = a.min_y[k];
                    mz[i] = a.min_z[k];
                } else {
                    mx[i] = 0.f;
                    my[i] = 0.f;
                    mz[i] = M0[i];
                }
                if (a.has_pre) {  // Eq. (4), (5) with the phase reduced in FP64
                    const double cyc = a.pre_cyc[0] * X[i] + a.pre_cyc[1] * Y[i] + a.pre_cyc[2] * Z[i] +
                                       df * a.pre_tau;
                    float s, c;
                    sincos_rev(cyc, &s, &c);
                    const float e2 = (float)exp(-a.pre_tau / t2);
                    const float e1 = (float)exp(-a.pre_tau / t1);
                    const float nx = e2 * (mx[i] * c + my[i] * s);
                    const float ny = e2 * (my[i] * c - mx[i] * s);
                    mx[i] = nx;
                    my[i] = ny;
                    mz[i] = fmaf(e1, mz[i] - M0[i], M0[i]);
                }
            } else {
                X[i] = Y[i] = Z[i] = 0.f;
                boff[i] = e1m[i] = e2m[i] = M0[i] = 0.f;
                mx[i] = my[i] = mz[i] = 0.f;
            }
        }

        int j = 0;
        for (int n = 0; n <= ns; ++n) {
            const int jend = n < ns ? sidx[n] - a.step_base : a.n_steps;
#pragma unroll 2
            for (; j < jend; ++j) {
                const StepW w = wave_ptr[j];
#pragma unroll
                for (int i = 0; i < kIso; ++i) {
                    const float bz = fmaf(w.gx, X[i], fmaf(w.gy, Y[i], fmaf(w.gz, Z[i], boff[i])));
                    float ca, cb;
                    if (HAS_B1) {
                        const float B2 = fmaf(bz, bz, w.b1sq);
                        rot_coeffs(B2, gdt, k2, ca, cb);
                        const float cx = w.b1i * mz[i] - bz * my[i];
                        const float cy = bz * mx[i] - w.b1r * mz[i];
                        const float cz = w.b1r * my[i] - w.b1i * mx[i];
                        const float d = fmaf(w.b1r, mx[i], fmaf(w.b1i, my[i], bz * mz[i]));
                        const float dx = fmaf(ca, cx, cb * fmaf(w.b1r, d, -B2 * mx[i]));
                        const float dy = fmaf(ca, cy, cb * fmaf(w.b1i, d, -B2 * my[i]));
                        const float dz = fmaf(ca, cz, cb * fmaf(bz, d, -B2 * mz[i]));
                        mx[i] += dx;
                        my[i] += dy;
                        mz[i] += dz;
                    } else {  // B = (0, 0, bz): rotation about z
                        const float B2 = bz * bz;
                        rot_coeffs(B2, gdt, k2, ca, cb);
                        const float p = ca * bz, r = cb * B2;
                        const float nx = fmaf(-p, my[i], fmaf(-r, mx[i], mx[i]));
                        const float ny = fmaf(p, mx[i], fmaf(-r, my[i], my[i]));
                        mx[i] = nx;
                        my[i] = ny;
                    }
                    mx[i] = fmaf(-e2m[i], mx[i], mx[i]);  // D: T2 decay, T1 recovery
                    my[i] = fmaf(-e2m[i], my[i], my[i]);
                    mz[i] = fmaf(e1m[i], M0[i] - mz[i], mz[i]);
                }
            }
            if (n < ns) {
                float vx = mx[0], vy = my[0];
#pragma unroll
                for (int i = 1; i < kIso; ++i) {
                    vx += mx[i];
                    vy += my[i];
                }
                vx = wave_sum_lane63(vx);
                vy = wave_sum_lane63(vy);
                if (lane == 63) {
                    float4 t = acc[wave * ns + n];
                    kahan_add(t.x, t.y, vx);
                    kahan_add(t.z, t.w, vy);
                    acc[wave * ns + n] = t;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kIso; ++i) {
            const int64_t k = base + (int64_t)i * kPlainBlock + tid;
            if (k < a.K) {
                a.mout_x[k] = mx[i];
                a.mout_y[k] = my[i];
                a.mout_z[k] = mz[i];
            }
        }
    }
    if (ns == 0) return;
    __syncthreads();
    for (int n = tid; n < ns; n += kPlainBlock) {
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const float4 t = acc[w * ns + n];
            re += (double)t.x - (double)t.y;
            im += (double)t.z - (double)t.w;
        }
        a.partial[(int64_t)blockIdx.x * ns + n] = make_double2(re, im);
    }
}

__global__ void k_plain_finalize(const double2 *__restrict__ partial, int nblk, int ns,
                                 double *__restrict__ sig) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= ns) return;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < nblk; ++b) {
        const double2 p = partial[(int64_t)b * ns + n];
        re += p.x;
        im += p.y;
    }
    sig[2 * n] += re;
    sig[2 * n + 1] += im;
}

int plain_grid(int64_t K) {
    const int64_t tiles = (K + kTile - 1) / kTile;
    const int64_t cap = 2048;  // 8 workgroups per CU on 256 CUs
    return (int)(tiles < cap ? (tiles > 0 ? tiles : 1) : cap);
}

hipError_t launch_plain(const PlainArgs &a, bool has_b1, int grid, hipStream_t st) {
    const size_t lds = sizeof(float4) * 4 * (size_t)a.n_samples;
    if (has_b1)
        hipLaunchKernelGGL(k_plain<true>, dim3(grid), dim3(kPlainBlock), lds, st, a);
    else
        hipLaunchKernelGGL(k_plain<false>, dim3(grid), dim3(kPlainBlock), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_plain_finalize(const double2 *partial, int nblk, int n_samples, double *sig,
                                 hipStream_t st) {
    if (n_samples <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_plain_finalize, dim3((n_samples + 255) / 256), dim3(256), 0, st, partial,
                       nblk, n_samples, sig);
    return hipGetLastError();
}

}  // namespace gbs
