// The conventional accelerated method on gfx950 (Sec. 2.2), the comparator
// of the grouped update.
//
// k_cached: one thread per isochromat.  In compose mode the thread multiplies
// its 3x4 homogeneous transition [A | b] (M' = A M + b M0) by D R for every
// raster step of the block in FP64 (Eq. 7 with U = D R of Eq. A1, A2; the
// step's waveform values are wave-uniform scalar loads), rounds it to FP32
// into the cache and applies it.  Later occurrences of the same waveform read
// the 48 cached bytes instead (dynamic caching).  The state between operations
// is FP64, 24 bytes per isochromat.
//
// k_direct_adc: Eq. (6) with Eq. (4), (5) evaluated for every (isochromat,
// sample) pair of a with-ADC block without RF.  Thread t of a workgroup owns
// sample t mod ns, and the slice t / ns of the isochromats when ns < 256.
// Isochromats pass through LDS in chunks of 256 and are read as broadcasts,
// so every thread keeps its sample's sum in registers and no cross-lane
// reduction runs per sample.  The phase is formed and reduced modulo one cycle
// in FP64 and evaluated with the hardware sin/cos; the T2 decay uses the
// hardware exp2.
#include "cached.hpp"
#include "consts.hpp"
#include "device_math.hpp"
#include "rotation.hpp"

namespace gbs {

constexpr int kCachedBlock = 256;
constexpr int kAdcBlock = 256;
constexpr int kAdcMaxGrid = 2048;  // 8 workgroups per CU on 256 CUs
constexpr double kLog2e = 1.44269504088896340736;

template <int MODE>
__global__ __launch_bounds__(kCachedBlock) void k_cached(CachedArgs a) {
    const int64_t k = (int64_t)blockIdx.x * kCachedBlock + threadIdx.x;
    if (k >= a.K) return;
    if (a.gate && *a.gate != a.gate_value) return;
    const int64_t K = a.K;
    const double m0 = a.ph.m0[k];
    double vx, vy, vz;
    if (a.s64_in) {
        vx = a.s64_in[k];
        vy = a.s64_in[K + k];
        vz = a.s64_in[2 * K + k];
    } else if (a.min_x) {
        vx = a.min_x[k];
        vy = a.min_y[k];
        vz = a.min_z[k];
    } else {
        vx = 0.0;
        vy = 0.0;
        vz = m0;
    }
    if (a.has_pre) {  // Eq. (4), (5); phase reduced modulo one cycle in FP64
        const double x = a.ph.x[k], y = a.ph.y[k], z = a.ph.z[k], df = a.ph.df[k];
        const double cyc = fma(a.pre_cyc[0], x, fma(a.pre_cyc[1], y, fma(a.pre_cyc[2], z, df * a.pre_tau)));
        double sn, cs;
        sincos(kTwoPi * (cyc - rint(cyc)), &sn, &cs);
        const double e2 = exp(-a.pre_tau / (double)a.ph.t2[k]);
        const double e1 = exp(-a.pre_tau / (double)a.ph.t1[k]);
        const double nx = e2 * (vx * cs + vy * sn);
        const double ny = e2 * (vy * cs - vx * sn);
        vx = nx;
        vy = ny;
        vz = m0 + (vz - m0) * e1;
    }
    if (MODE == kCacheApply) {
        const float4 r0 = a.cache[k], r1 = a.cache[K + k], r2 = a.cache[2 * K + k];
        const double nx = fma((double)r0.x, vx, fma((double)r0.y, vy, fma((double)r0.z, vz, (double)r0.w * m0)));
        const double ny = fma((double)r1.x, vx, fma((double)r1.y, vy, fma((double)r1.z, vz, (double)r1.w * m0)));
        const double nz = fma((double)r2.x, vx, fma((double)r2.y, vy, fma((double)r2.z, vz, (double)r2.w * m0)));
        vx = nx;
        vy = ny;
        vz = nz;
    } else if (MODE == kCacheCompose) {
        const double X = a.ph.x[k], Y = a.ph.y[k], Z = a.ph.z[k];
        const double boff = (double)a.ph.df[k] / kGammaBar;  // off-resonance as a field (T)
        const double t1 = a.ph.t1[k], t2 = a.ph.t2[k];
        const double e1 = exp(-a.dt / t1), e2 = exp(-a.dt / t2), e1m = -expm1(-a.dt / t1);
        const double gdt = a.gdt, k2 = gdt * gdt;
        // T = [A | b], starting from the identity map
        double T[3][4] = {{1.0, 0.0, 0.0, 0.0}, {0.0, 1.0, 0.0, 0.0}, {0.0, 0.0, 1.0, 0.0}}, U[3][4];
        const StepW *__restrict__ wave = a.wave;
        // V = (D R)_j V0 for raster step j, then the T1 recovery toward M0
        auto step = [&](const double (&V0)[3][4], double (&V)[3][4], int j) {
            const StepW w = wave[j];
            const double bx = w.b1r, by = w.b1i;
            const double bz = fma((double)w.gx, X, fma((double)w.gy, Y, fma((double)w.gz, Z, boff)));
            const double B2 = fma(bx, bx, fma(by, by, bz * bz));
            double ca, cb;  // R = (1 - cb |B|^2) I + ca [B]x + cb B B^T
            rot_coeffs(B2, gdt, k2, ca, cb);
            const double c0 = fma(-cb, B2, 1.0);
            const double qx = cb * bx, qy = cb * by, qz = cb * bz;
            const double pxy = qx * by, pxz = qx * bz, pyz = qy * bz;
            const double sx = ca * bx, sy = ca * by, sz = ca * bz;
            // rows of D R: transverse rows decay by E2, the z row by E1
            const double r00 = e2 * fma(qx, bx, c0), r01 = e2 * (pxy - sz), r02 = e2 * (pxz + sy);
            const double r10 = e2 * (pxy + sz), r11 = e2 * fma(qy, by, c0), r12 = e2 * (pyz - sx);
            const double r20 = e1 * (pxz - sy), r21 = e1 * (pyz + sx), r22 = e1 * fma(qz, bz, c0);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double u0 = V0[0][c], u1 = V0[1][c], u2 = V0[2][c];
                V[0][c] = fma(r00, u0, fma(r01, u1, r02 * u2));
                V[1][c] = fma(r10, u0, fma(r11, u1, r12 * u2));
                V[2][c] = fma(r20, u0, fma(r21, u1, r22 * u2));
            }
            V[2][3] += e1m;
        };
        // two steps per iteration, T -> U -> T, so that the loop carries no
        // register copies of the twelve entries
        int j = 0;
        for (; j + 1 < a.n_steps; j += 2) {
            step(T, U, j);
            step(U, T, j + 1);
        }
        if (j < a.n_steps) {
            step(T, U, j);
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) T[r][c] = U[r][c];
        }
        a.cache[k] = make_float4((float)T[0][0], (float)T[0][1], (float)T[0][2], (float)T[0][3]);
        a.cache[K + k] = make_float4((float)T[1][0], (float)T[1][1], (float)T[1][2], (float)T[1][3]);
        a.cache[2 * K + k] = make_float4((float)T[2][0], (float)T[2][1], (float)T[2][2], (float)T[2][3]);
        const double nx = fma(T[0][0], vx, fma(T[0][1], vy, fma(T[0][2], vz, T[0][3] * m0)));
        const double ny = fma(T[1][0], vx, fma(T[1][1], vy, fma(T[1][2], vz, T[1][3] * m0)));
        const double nz = fma(T[2][0], vx, fma(T[2][1], vy, fma(T[2][2], vz, T[2][3] * m0)));
        vx = nx;
        vy = ny;
        vz = nz;
    }
    if (a.s64_out) {
        a.s64_out[k] = vx;
        a.s64_out[K + k] = vy;
        a.s64_out[2 * K + k] = vz;
    } else {
        a.mout_x[k] = (float)vx;
        a.mout_y[k] = (float)vy;
        a.mout_z[k] = (float)vz;
    }
}

template <bool COILS>
__global__ __launch_bounds__(kAdcBlock) void k_direct_adc(DirectAdcArgs a) {
    constexpr int MC = COILS ? kMaxCoils : 1;
    __shared__ double4 pos[kAdcBlock];  // x, y, z, df
    __shared__ float4 mag[kAdcBlock];   // Mx, My, -log2(e) / T2, 0
    __shared__ float2 sen[MC][kAdcBlock];  // S(k, p) of the chunk (coils only)
    __shared__ double2 red[kAdcBlock];
    const int t = threadIdx.x;
    const int ns = a.n_samples;
    const int P = COILS ? a.n_coils : 1;
    const int G = kAdcBlock / ns;  // isochromat slices per chunk
    const int cnt = kAdcBlock / G;
    const int n = t % ns, g = t / ns;
    const bool active = g < G;
    const double4 c = active ? a.samp[n] : make_double4(0.0, 0.0, 0.0, 0.0);
    const float tau = (float)c.w;
    const int64_t K = a.K;
    double acc_re[MC], acc_im[MC];
#pragma unroll
    for (int p = 0; p < MC; ++p) acc_re[p] = acc_im[p] = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * kAdcBlock; base < K; base += (int64_t)gridDim.x * kAdcBlock) {
        const int64_t k = base + t;
        double4 q0 = make_double4(0.0, 0.0, 0.0, 0.0);
        float4 m = make_float4(0.f, 0.f, 0.f, 0.f);  // padding slots add nothing
        if (k < K) {
            q0 = make_double4(a.ph.x[k], a.ph.y[k], a.ph.z[k], a.ph.df[k]);
            float mx = 0.f, my = 0.f;
            if (a.s64_in) {
                mx = (float)a.s64_in[k];
                my = (float)a.s64_in[K + k];
            } else if (a.min_x) {
                mx = a.min_x[k];
                my = a.min_y[k];
            }
            m = make_float4(mx, my, (float)(-kLog2e / (double)a.ph.t2[k]), 0.f);
        }
        __syncthreads();  // the previous chunk has been read
        pos[t] = q0;
        mag[t] = m;
        if (COILS) {
#pragma unroll
            for (int p = 0; p < MC; ++p)
                if (p < P) sen[p][t] = k < K ? make_float2(a.coil_re[p * K + k], a.coil_im[p * K + k])
                                             : make_float2(0.f, 0.f);
        }
        __syncthreads();
        if (active) {
            float sr[MC], si[MC];
#pragma unroll
            for (int p = 0; p < MC; ++p) sr[p] = si[p] = 0.f;
            auto add = [&](int j) {
                const double4 q = pos[j];
                const float4 v = mag[j];
                const double cyc = fma(c.x, q.x, fma(c.y, q.y, fma(c.z, q.z, c.w * q.w)));
                float s, co;
                sincos_rev(cyc, &s, &co);
                const float e = __builtin_amdgcn_exp2f(tau * v.z);  // exp(-tau / T2)
                // (Mx + i My) exp(-i 2 pi cyc)
                const float tr = e * fmaf(v.x, co, v.y * s), ti = e * fmaf(v.y, co, -v.x * s);
                if (COILS) {
#pragma unroll
                    for (int p = 0; p < MC; ++p)
                        if (p < P) {
                            const float2 w = sen[p][j];
                            sr[p] = fmaf(tr, w.x, fmaf(-ti, w.y, sr[p]));
                            si[p] = fmaf(tr, w.y, fmaf(ti, w.x, si[p]));
                        }
                } else {
                    sr[0] += tr;
                    si[0] += ti;
                }
            };
            // slice g takes chunk entries g, g + G, ...: cnt of them (a
            // wave-uniform count), and one more when 256 is not a multiple of G
#pragma unroll 4
            for (int i = 0; i < cnt; ++i) add(g + i * G);
            if (g + cnt * G < kAdcBlock) add(g + cnt * G);
#pragma unroll
            for (int p = 0; p < MC; ++p) {
                acc_re[p] += sr[p];
                acc_im[p] += si[p];
            }
        }
    }
#pragma unroll
    for (int p = 0; p < MC; ++p) {
        if (p >= P) break;
        if (p > 0) __syncthreads();  // the previous coil's sums have been read
        red[t] = make_double2(acc_re[p], acc_im[p]);
        __syncthreads();
        if (t < ns) {
            double re = 0.0, im = 0.0;
            for (int q = 0; q < G; ++q) {
                re += red[q * ns + t].x;
                im += red[q * ns + t].y;
            }
            a.partial[((int64_t)p * gridDim.x + blockIdx.x) * ns + t] = make_double2(re, im);
        }
    }
}

hipError_t launch_cached(const CachedArgs &a, int mode, hipStream_t st) {
    const int64_t blocks = (a.K + kCachedBlock - 1) / kCachedBlock;
    if (blocks <= 0) return hipSuccess;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(kCachedBlock);
    switch (mode) {
        case kCacheMap: hipLaunchKernelGGL(k_cached<kCacheMap>, grid, block, 0, st, a); break;
        case kCacheApply: hipLaunchKernelGGL(k_cached<kCacheApply>, grid, block, 0, st, a); break;
        case kCacheCompose: hipLaunchKernelGGL(k_cached<kCacheCompose>, grid, block, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int direct_adc_grid(int64_t K) {
    const int64_t chunks = (K + kAdcBlock - 1) / kAdcBlock;
    return (int)(chunks < kAdcMaxGrid ? (chunks > 0 ? chunks : 1) : kAdcMaxGrid);
}

hipError_t launch_direct_adc(const DirectAdcArgs &a, int grid, hipStream_t st) {
    if (a.n_samples < 1 || a.n_samples > kAdcBlock || grid < 1 || grid > kAdcMaxGrid) return hipErrorInvalidValue;
    if (a.coil_re) {
        if (!a.coil_im || a.n_coils < 1 || a.n_coils > kMaxCoils) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_direct_adc<true>, dim3(grid), dim3(kAdcBlock), 0, st, a);
    } else {
        hipLaunchKernelGGL(k_direct_adc<false>, dim3(grid), dim3(kAdcBlock), 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace gbs
