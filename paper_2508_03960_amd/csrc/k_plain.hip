// Plain per-isochromat stepping on gfx950 (the conventional method that the
// grouped update is measured against, Sec. 2.2).
//
// One thread carries kIso isochromats in registers through every raster step
// of a block: U = D R (Eq. 2, Eq. A1, Eq. A2).  The waveform value of a step
// is the same for every lane, so it is one scalar load per step.
//
// The step is applied in increment form:
//   R M = M + a (B x M) + b (B (B . M) - |B|^2 M),
//   a = sin(theta)/|B|,  b = (1 - cos theta)/|B|^2,  theta = -gamma |B| dt,
// with a, b from their power series in q = theta^2 (no sqrt, no division, and
// R = I falls out at B = 0); relaxation as M -= (1 - E) M with
// 1 - E = -expm1(-dt/T) computed once per isochromat.
//
// The arithmetic type R is double by default and float on request.  In float
// the rounded per-step coefficients bias every step of a constant-gradient
// readout the same way (about 1e-8 per step), which over tens of thousands of
// steps exceeds 1e-5; the double version keeps the state exact to ~1e-12 at
// the same FMA rate (packed FP32 is not used on this target).
//
// ADC samples (Eq. 6): at each sample boundary a wavefront sums its lanes with
// DPP, lane 63 adds the wave total into a per-wave LDS accumulator
// (compensated FP32, or FP64); at the end each workgroup writes one FP64
// partial per sample, and a finalize kernel (one workgroup per sample) adds
// the partials in a fixed order.
#include "device_math.hpp"
#include "kernels.hpp"
#include "plain_coils.hpp"
#include "rotation.hpp"

namespace gbs {

constexpr int kPlainBlock = 256;
constexpr int kIso = 2;
constexpr int kTile = kPlainBlock * kIso;

// Per-wave ADC accumulator in LDS: compensated FP32, or plain FP64.
template <typename R>
struct SampleAcc;

template <>
struct SampleAcc<float> {
    float4 v;  // (sum re, comp re, sum im, comp im)
    static __device__ __forceinline__ void add(SampleAcc &a, float x, float y) {
        kahan_add(a.v.x, a.v.y, x);
        kahan_add(a.v.z, a.v.w, y);
    }
    __device__ __forceinline__ double re() const { return (double)v.x - (double)v.y; }
    __device__ __forceinline__ double im() const { return (double)v.z - (double)v.w; }
    static __device__ __forceinline__ float wave_sum(float x) { return wave_sum_lane63(x); }
};

template <>
struct SampleAcc<double> {
    double2 v;
    static __device__ __forceinline__ void add(SampleAcc &a, double x, double y) {
        a.v.x += x;
        a.v.y += y;
    }
    __device__ __forceinline__ double re() const { return v.x; }
    __device__ __forceinline__ double im() const { return v.y; }
    static __device__ __forceinline__ double wave_sum(double x) { return wave_sum_lane63_f64(x); }
};

template <typename R>
__device__ __forceinline__ R fmaR(R a, R b, R c);
template <>
__device__ __forceinline__ float fmaR<float>(float a, float b, float c) { return fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fmaR<double>(double a, double b, double c) { return fma(a, b, c); }

template <typename R, bool HAS_B1, bool COILS>
__global__ __launch_bounds__(kPlainBlock) void k_plain(PlainArgs a, PlainCoils cl) {
    using Acc = SampleAcc<R>;
    constexpr int MC = COILS ? kPlainMaxCoils : 1;
    extern __shared__ char lds_raw[];
    Acc *acc = reinterpret_cast<Acc *>(lds_raw);  // [4 waves][n_samples][coils]
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int ns = a.n_samples;
    const int P = COILS ? cl.n : 1;
    for (int i = tid; i < 4 * ns * P; i += kPlainBlock) acc[i] = Acc{};
    __syncthreads();
    const R gdt = (R)a.gdt;
    const R k2 = gdt * gdt;
    const StepW *__restrict__ wave_ptr = a.wave;
    const int32_t *__restrict__ sidx = a.sidx;

    for (int64_t base = (int64_t)blockIdx.x * kTile; base < a.K; base += (int64_t)gridDim.x * kTile) {
        R X[kIso], Y[kIso], Z[kIso], boff[kIso], e1m[kIso], e2m[kIso], M0[kIso];
        R mx[kIso], my[kIso], mz[kIso];
        float csr[MC][kIso], csi[MC][kIso];  // coil sensitivities of the thread's isochromats
#pragma unroll
        for (int p = 0; p < MC; ++p)
#pragma unroll
            for (int i = 0; i < kIso; ++i) {
                const int64_t k = base + (int64_t)i * kPlainBlock + tid;
                const bool use = COILS && p < P && k < a.K;
                csr[p][i] = use ? cl.re[p * cl.stride + k] : 0.f;
                csi[p][i] = use ? cl.im[p * cl.stride + k] : 0.f;
            }
#pragma unroll
        for (int i = 0; i < kIso; ++i) {
            const int64_t k = base + (int64_t)i * kPlainBlock + tid;
            if (k < a.K) {
                const double x = a.ph.x[k], y = a.ph.y[k], z = a.ph.z[k];
                const double t1 = a.ph.t1[k], t2 = a.ph.t2[k], df = a.ph.df[k];
                const double m0 = a.ph.m0[k];
                double vx = 0.0, vy = 0.0, vz = m0;
                if (a.min64_x) {
                    vx = a.min64_x[k];
                    vy = a.min64_y[k];
                    vz = a.min64_z[k];
                } else if (a.min_x) {
                    vx = a.min_x[k];
                    vy = a.min_y[k];
                    vz = a.min_z[k];
                }
                if (a.has_pre) {  // Eq. (4), (5); phase reduced modulo one cycle in FP64
                    const double cyc = a.pre_cyc[0] * x + a.pre_cyc[1] * y + a.pre_cyc[2] * z + df * a.pre_tau;
                    double sn, cs;
                    sincos(kTwoPi * (cyc - rint(cyc)), &sn, &cs);
                    const double e2 = exp(-a.pre_tau / t2), e1 = exp(-a.pre_tau / t1);
                    const double nx = e2 * (vx * cs + vy * sn);
                    const double ny = e2 * (vy * cs - vx * sn);
                    vx = nx;
                    vy = ny;
                    vz = m0 + (vz - m0) * e1;
                }
                X[i] = (R)x;
                Y[i] = (R)y;
                Z[i] = (R)z;
                M0[i] = (R)m0;
                boff[i] = (R)(df / kGammaBar);
                e1m[i] = (R)(-expm1(-a.dt / t1));
                e2m[i] = (R)(-expm1(-a.dt / t2));
                mx[i] = (R)vx;
                my[i] = (R)vy;
                mz[i] = (R)vz;
            } else {
                X[i] = Y[i] = Z[i] = R(0);
                boff[i] = e1m[i] = e2m[i] = M0[i] = R(0);
                mx[i] = my[i] = mz[i] = R(0);
            }
        }

        int j = 0;
        for (int n = 0; n <= ns; ++n) {
            const int jend = n < ns ? sidx[n] - a.step_base : a.n_steps;
#pragma unroll 2
            for (; j < jend; ++j) {
                const StepW w = wave_ptr[j];
                const R b1r = (R)w.b1r, b1i = (R)w.b1i, b1sq = (R)w.b1sq;
                const R gx = (R)w.gx, gy = (R)w.gy, gz = (R)w.gz;
#pragma unroll
                for (int i = 0; i < kIso; ++i) {
                    const R bz = fmaR(gx, X[i], fmaR(gy, Y[i], fmaR(gz, Z[i], boff[i])));
                    R ca, cb;
                    if (HAS_B1) {
                        const R B2 = fmaR(bz, bz, b1sq);
                        rot_coeffs<R>(B2, gdt, k2, ca, cb);
                        const R cx = b1i * mz[i] - bz * my[i];
                        const R cy = bz * mx[i] - b1r * mz[i];
                        const R cz = b1r * my[i] - b1i * mx[i];
                        const R d = fmaR(b1r, mx[i], fmaR(b1i, my[i], bz * mz[i]));
                        const R dx = fmaR(ca, cx, cb * fmaR(b1r, d, -B2 * mx[i]));
                        const R dy = fmaR(ca, cy, cb * fmaR(b1i, d, -B2 * my[i]));
                        const R dz = fmaR(ca, cz, cb * fmaR(bz, d, -B2 * mz[i]));
                        mx[i] += dx;
                        my[i] += dy;
                        mz[i] += dz;
                    } else {  // B = (0, 0, bz): rotation about z
                        const R B2 = bz * bz;
                        rot_coeffs<R>(B2, gdt, k2, ca, cb);
                        const R p = ca * bz, r = cb * B2;
                        const R nx = fmaR(-p, my[i], fmaR(-r, mx[i], mx[i]));
                        const R ny = fmaR(p, mx[i], fmaR(-r, my[i], my[i]));
                        mx[i] = nx;
                        my[i] = ny;
                    }
                    mx[i] = fmaR(-e2m[i], mx[i], mx[i]);  // D: T2 decay, T1 recovery
                    my[i] = fmaR(-e2m[i], my[i], my[i]);
                    mz[i] = fmaR(e1m[i], M0[i] - mz[i], mz[i]);
                }
            }
            if (n < ns && COILS) {  // one sum per coil: S(k, p) (Mx + i My)
#pragma unroll
                for (int p = 0; p < MC; ++p) {
                    if (p >= P) break;
                    R vx = R(0), vy = R(0);
#pragma unroll
                    for (int i = 0; i < kIso; ++i) {
                        const R sr = (R)csr[p][i], si = (R)csi[p][i];
                        vx += mx[i] * sr - my[i] * si;
                        vy += mx[i] * si + my[i] * sr;
                    }
                    vx = Acc::wave_sum(vx);
                    vy = Acc::wave_sum(vy);
                    if (lane == 63) Acc::add(acc[(wave * ns + n) * P + p], vx, vy);
                }
            } else if (n < ns) {
                R vx = mx[0], vy = my[0];
#pragma unroll
                for (int i = 1; i < kIso; ++i) {
                    vx += mx[i];
                    vy += my[i];
                }
                vx = Acc::wave_sum(vx);
                vy = Acc::wave_sum(vy);
                if (lane == 63) Acc::add(acc[wave * ns + n], vx, vy);
            }
        }
#pragma unroll
        for (int i = 0; i < kIso; ++i) {
            const int64_t k = base + (int64_t)i * kPlainBlock + tid;
            if (k < a.K) {
                if (a.mout_x) {
                    a.mout_x[k] = (float)mx[i];
                    a.mout_y[k] = (float)my[i];
                    a.mout_z[k] = (float)mz[i];
                }
                if (a.mout64_x) {
                    a.mout64_x[k] = (double)mx[i];
                    a.mout64_y[k] = (double)my[i];
                    a.mout64_z[k] = (double)mz[i];
                }
            }
        }
    }
    if (ns == 0) return;
    __syncthreads();
    for (int idx = tid; idx < ns * P; idx += kPlainBlock) {  // partials [coil][workgroup][sample]
        const int n = idx / P, p = idx - n * P;
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            re += acc[(w * ns + n) * P + p].re();
            im += acc[(w * ns + n) * P + p].im();
        }
        a.partial[((int64_t)p * gridDim.x + blockIdx.x) * ns + n] = make_double2(re, im);
    }
}

// One workgroup per sample: thread t adds partials t, t + 256, ... in order,
// then a fixed LDS tree adds the 256 thread sums (the same order every run).
__global__ __launch_bounds__(256) void k_plain_finalize(const double2 *__restrict__ partial, int nblk, int ns,
                                                        double *__restrict__ sig) {
    __shared__ double2 red[256];
    const int n = blockIdx.x, t = threadIdx.x;
    double re = 0.0, im = 0.0;
    for (int b = t; b < nblk; b += 256) {
        const double2 p = partial[(int64_t)b * ns + n];
        re += p.x;
        im += p.y;
    }
    red[t] = make_double2(re, im);
    __syncthreads();
#pragma unroll
    for (int w = 128; w >= 1; w /= 2) {
        if (t < w) {
            red[t].x += red[t + w].x;
            red[t].y += red[t + w].y;
        }
        __syncthreads();
    }
    if (t == 0) {
        sig[2 * n] += red[0].x;
        sig[2 * n + 1] += red[0].y;
    }
}

int plain_grid(int64_t K) {
    const int64_t tiles = (K + kTile - 1) / kTile;
    const int64_t cap = 2048;  // 8 workgroups per CU on 256 CUs
    return (int)(tiles < cap ? (tiles > 0 ? tiles : 1) : cap);
}

hipError_t launch_plain(const PlainArgs &a, bool has_b1, bool fp32, int grid, hipStream_t st) {
    const size_t lds = 16 * 4 * (size_t)a.n_samples;  // both accumulator types are 16 bytes
    const PlainCoils none{nullptr, nullptr, 0, 1};
    if (fp32) {
        if (has_b1)
            hipLaunchKernelGGL((k_plain<float, true, false>), dim3(grid), dim3(kPlainBlock), lds, st, a, none);
        else
            hipLaunchKernelGGL((k_plain<float, false, false>), dim3(grid), dim3(kPlainBlock), lds, st, a, none);
    } else {
        if (has_b1)
            hipLaunchKernelGGL((k_plain<double, true, false>), dim3(grid), dim3(kPlainBlock), lds, st, a, none);
        else
            hipLaunchKernelGGL((k_plain<double, false, false>), dim3(grid), dim3(kPlainBlock), lds, st, a, none);
    }
    return hipGetLastError();
}

hipError_t launch_plain_coils(const PlainArgs &a, const PlainCoils &c, bool has_b1, bool fp32, int grid,
                              hipStream_t st) {
    if (!c.re || !c.im || c.n < 1 || c.n > kPlainMaxCoils || a.n_samples * c.n > 256) return hipErrorInvalidValue;
    const size_t lds = 16 * 4 * (size_t)a.n_samples * (size_t)c.n;
    if (fp32) {
        if (has_b1)
            hipLaunchKernelGGL((k_plain<float, true, true>), dim3(grid), dim3(kPlainBlock), lds, st, a, c);
        else
            hipLaunchKernelGGL((k_plain<float, false, true>), dim3(grid), dim3(kPlainBlock), lds, st, a, c);
    } else {
        if (has_b1)
            hipLaunchKernelGGL((k_plain<double, true, true>), dim3(grid), dim3(kPlainBlock), lds, st, a, c);
        else
            hipLaunchKernelGGL((k_plain<double, false, true>), dim3(grid), dim3(kPlainBlock), lds, st, a, c);
    }
    return hipGetLastError();
}

hipError_t launch_plain_finalize(const double2 *partial, int nblk, int n_samples, double *sig,
                                 hipStream_t st) {
    if (n_samples <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_plain_finalize, dim3(n_samples), dim3(256), 0, st, partial, nblk, n_samples, sig);
    return hipGetLastError();
}

}  // namespace gbs
