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
// The state and every coefficient are FP64.  In FP32 the rounded per-step
// coefficients turn the same rounding into an angle error at every step of a
// constant-gradient readout (about 1e-8 of the angle per step), which adds up
// coherently over tens of thousands of steps to far more than 1e-5 of M;
// removing that with compensated FP32 arithmetic (double-float coefficients
// and a compensated state) costs more instructions than FP64, which issues at
// the non-packed FP32 rate on this target.
//
// ADC samples (Eq. 6): at each sample boundary a wavefront sums its lanes with
// DPP, lane 63 adds the wave total into a per-wave FP64 LDS accumulator;
// at the end each workgroup writes one FP64
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

// Per-wave ADC accumulator in LDS (FP64).
struct SampleAcc {
    double2 v;
    static __device__ __forceinline__ void add(SampleAcc &a, double x, double y) {
        a.v.x += x;
        a.v.y += y;
    }
    __device__ __forceinline__ double re() const { return v.x; }
    __device__ __forceinline__ double im() const { return v.y; }
    static __device__ __forceinline__ double wave_sum(double x) { return wave_sum_lane63_f64(x); }
};

template <bool HAS_B1, bool COILS>
__global__ __launch_bounds__(kPlainBlock) void k_plain(PlainArgs a, PlainCoils cl) {
    using R = double;
    using Acc = SampleAcc;
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
    const R gdt = a.gdt;
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
                X[i] = x;
                Y[i] = y;
                Z[i] = z;
                M0[i] = m0;
                boff[i] = df / kGammaBar;
                e1m[i] = -expm1(-a.dt / t1);
                e2m[i] = -expm1(-a.dt / t2);
                mx[i] = vx;
                my[i] = vy;
                mz[i] = vz;
            } else {
                X[i] = Y[i] = Z[i] = 0.0;
                boff[i] = e1m[i] = e2m[i] = M0[i] = 0.0;
                mx[i] = my[i] = mz[i] = 0.0;
            }
        }

        int j = 0;
        for (int n = 0; n <= ns; ++n) {
            const int jend = n < ns ? sidx[n] - a.step_base : a.n_steps;
            // not unrolled: the Horner steps are inline asm, which the compiler
            // treats as convergent; at 124-126 VGPRs four waves share a SIMD
            for (; j < jend; ++j) {
                const StepW w = wave_ptr[j];
                const R b1r = w.b1r, b1i = w.b1i, b1sq = w.b1sq;
                const R gx = w.gx, gy = w.gy, gz = w.gz;
#pragma unroll
                for (int i = 0; i < kIso; ++i) {
                    const R bz = fma(gx, X[i], fma(gy, Y[i], fma(gz, Z[i], boff[i])));
                    R ca, cb;
                    if (HAS_B1) {
                        const R B2 = fma(bz, bz, b1sq);
                        rot_coeffs(B2, gdt, k2, ca, cb);
                        const R cx = b1i * mz[i] - bz * my[i];
                        const R cy = bz * mx[i] - b1r * mz[i];
                        const R cz = b1r * my[i] - b1i * mx[i];
                        const R d = fma(b1r, mx[i], fma(b1i, my[i], bz * mz[i]));
                        const R dx = fma(ca, cx, cb * fma(b1r, d, -B2 * mx[i]));
                        const R dy = fma(ca, cy, cb * fma(b1i, d, -B2 * my[i]));
                        const R dz = fma(ca, cz, cb * fma(bz, d, -B2 * mz[i]));
                        mx[i] += dx;
                        my[i] += dy;
                        mz[i] += dz;
                    } else {  // B = (0, 0, bz): rotation about z
                        const R B2 = bz * bz;
                        rot_coeffs(B2, gdt, k2, ca, cb);
                        const R p = ca * bz, r = cb * B2;
                        const R nx = fma(-p, my[i], fma(-r, mx[i], mx[i]));
                        const R ny = fma(p, mx[i], fma(-r, my[i], my[i]));
                        mx[i] = nx;
                        my[i] = ny;
                    }
                    mx[i] = fma(-e2m[i], mx[i], mx[i]);  // D: T2 decay, T1 recovery
                    my[i] = fma(-e2m[i], my[i], my[i]);
                    mz[i] = fma(e1m[i], M0[i] - mz[i], mz[i]);
                }
            }
            if (n < ns && COILS) {  // one sum per coil: S(k, p) (Mx + i My)
#pragma unroll
                for (int p = 0; p < MC; ++p) {
                    if (p >= P) break;
                    R vx = 0.0, vy = 0.0;
#pragma unroll
                    for (int i = 0; i < kIso; ++i) {
                        const R sr = csr[p][i], si = csi[p][i];
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

hipError_t launch_plain(const PlainArgs &a, bool has_b1, int grid, hipStream_t st) {
    const size_t lds = sizeof(SampleAcc) * 4 * (size_t)a.n_samples;
    const PlainCoils none{nullptr, nullptr, 0, 1};
    if (has_b1)
        hipLaunchKernelGGL((k_plain<true, false>), dim3(grid), dim3(kPlainBlock), lds, st, a, none);
    else
        hipLaunchKernelGGL((k_plain<false, false>), dim3(grid), dim3(kPlainBlock), lds, st, a, none);
    return hipGetLastError();
}

hipError_t launch_plain_coils(const PlainArgs &a, const PlainCoils &c, bool has_b1, int grid, hipStream_t st) {
    if (!c.re || !c.im || c.n < 1 || c.n > kPlainMaxCoils || a.n_samples * c.n > 256) return hipErrorInvalidValue;
    const size_t lds = sizeof(SampleAcc) * 4 * (size_t)a.n_samples * (size_t)c.n;
    if (has_b1)
        hipLaunchKernelGGL((k_plain<true, true>), dim3(grid), dim3(kPlainBlock), lds, st, a, c);
    else
        hipLaunchKernelGGL((k_plain<false, true>), dim3(grid), dim3(kPlainBlock), lds, st, a, c);
    return hipGetLastError();
}

hipError_t launch_plain_finalize(const double2 *partial, int nblk, int n_samples, double *sig,
                                 hipStream_t st) {
    if (n_samples <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_plain_finalize, dim3(n_samples), dim3(256), 0, st, partial, nblk, n_samples, sig);
    return hipGetLastError();
}

}  // namespace gbs
