// Reverse-mode (adjoint) Bloch simulation for gfx950: the gradient of
// L = sum_n (w_re[n] Re A_n + w_im[n] Im A_n) with respect to the samples of
// a parameter RF pulse and per-class T1, T2.  One isochromat per thread,
// FP32 state, FP64 accumulation of sums over isochromats.
//
// Compensated FP32 state.  A raster step changes M by a small increment
// (relaxation by dt/T of M, rotation by |w| ~ 1e-2); added to M in FP32,
// most of such an increment is rounded away, and the same way at every step
// while M changes slowly: a coherent bias that reached 4e-4 of M over the
// 8-TR workload.  So M and the adjoint state lambda are carried as FP32
// pairs (hi, lo): each op forms its increment from hi, and a two-sum adds
// increment + lo to hi, keeping the rounding error in lo.  Relaxation blocks
// form cos as 1 - c1 and sin as s + sl from an FP64 sincos, and E2 as 1 - om2,
// so their coefficients carry no rounding that repeats across identical
// blocks.  Checkpoints hold hi; a recomputed segment starts with lo = 0.
//
//  k_adj_forward   plain stepping (Eq. 2 with U = D R of Eq. A1, A2; Eq. 4, 5
//                  for relaxation blocks), the samples of Eq. 6, and the state
//                  at every `every`-th op boundary (checkpoints, SoA in HBM).
//  k_adj_backward  segments in reverse: from each checkpoint the segment is
//                  stepped again, keeping a sub-checkpoint every 8 ops in
//                  HBM; each 8-op sub-segment is stepped once more with its
//                  rotated states in registers and then walked backward:
//                      lambda_p = (D_p R_p)^T lambda_{p+1} + cotangent at p.
//  k_adj_finalize  sums the per-workgroup partials in FP64.
//
// Derivatives of one raster step M' = D R(w) M + (1 - E1) M0 e_z, with the
// rotation vector w = -2 pi gamma_bar dt B (R = exp([w]x), Eq. A2), v = R M
// and mu = D lambda':
//   dL/dw = J^T (v x mu),  J^T = I - C [w]x + D3 [w]x^2        (SO(3) Jacobian)
//   dL/dB1x = -2 pi gamma_bar dt (dL/dw)_x,   dL/dB1y likewise,
//   dL/dT2 += (lambda'_x M'_x + lambda'_y M'_y) dt / T2^2,
//   dL/dT1 += lambda'_z (M'_z - M0) dt / T1^2,
// with S = sin t / t, C = (1 - cos t) / t^2, D3 = (t - sin t) / t^3, t = |w|.
// A relaxation block is a z rotation by the phase of Eq. 4 and the decay of
// Eq. 4, 5 over tau: the same T1, T2 terms with dt -> tau.
#include "adj.hpp"
#include "consts.hpp"
#include "device_math.hpp"

namespace gbs {

// S, C, D3 of t = sqrt(q) from their Taylor series, terms k = 0 .. N:
//   S = sum_k (-q)^k / (2k+1)!,  C = sum_k (-q)^k / (2k+2)!,
//   D3 = sum_k (-q)^k / (2k+3)!.
template <int N>
__device__ __forceinline__ void rot_series(float q, float &S, float &C, float &D3) {
    // 1/k! for k = 0 .. 21
    constexpr float f[22] = {1.f, 1.f, 5.0e-1f, 1.6666666666666666e-1f, 4.1666666666666664e-2f,
                             8.3333333333333332e-3f, 1.3888888888888889e-3f, 1.9841269841269841e-4f,
                             2.4801587301587302e-5f, 2.7557319223985893e-6f, 2.7557319223985888e-7f,
                             2.5052108385441720e-8f, 2.0876756987868100e-9f, 1.6059043836821613e-10f,
                             1.1470745597729725e-11f, 7.6471637318198164e-13f, 4.7794773323873853e-14f,
                             2.8114572543455206e-15f, 1.5619206968586225e-16f, 8.2206352466243295e-18f,
                             4.1103176233121648e-19f, 1.9572941063391263e-20f};
    static_assert(2 * N + 3 < 22, "series length");
    float s = f[2 * N + 1], c = f[2 * N + 2], d = f[2 * N + 3];
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
        s = f[2 * k + 1] - q * s;
        c = f[2 * k + 2] - q * c;
        d = f[2 * k + 3] - q * d;
    }
    S = s;
    C = c;
    D3 = d;
}

// The series' length follows q: below q = 1/16 five terms leave out at most
// q^5 / 11! < 2.4e-14 (relative), below q = 4 nine terms at most
// 4^9 / 19! < 3e-12; larger angles take sqrt and sincos.  Raster steps
// rotate by far less than a quarter radian, so the short branch is the one
// taken.
__device__ __forceinline__ void rot_coeffs(float q, float &S, float &C, float &D3) {
    if (q < 0.0625f) {
        rot_series<4>(q, S, C, D3);
    } else if (q < 4.f) {
        rot_series<8>(q, S, C, D3);
    } else {
        const float t = sqrtf(q);
        float sn, cs;
        sincosf(t, &sn, &cs);
        S = sn / t;
        C = (1.f - cs) / q;
        D3 = (t - sn) / (q * t);
    }
}

// Op descriptors, the parameter pulse, the sample lists and the signal
// cotangent are read-only during a launch and indexed by wave-uniform values:
// they are read through the constant address space, so that they arrive in
// scalar registers instead of through vector loads the op loop must wait for.
typedef const __attribute__((address_space(4))) uint64_t *const_u64_ptr;
static_assert(sizeof(AdjOp) % 8 == 0, "AdjOp is read as 64-bit words");

__device__ __forceinline__ AdjOp load_op(const AdjOp *ops, int p) {
    uint64_t w[sizeof(AdjOp) / 8];
    const const_u64_ptr q = (const_u64_ptr)(ops + p);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(AdjOp) / 8); ++i) w[i] = q[i];
    AdjOp r;
    __builtin_memcpy(&r, w, sizeof(AdjOp));
    return r;
}

// Plain-old-data element i of p, as 64-bit (or one 32-bit) scalar words.
template <typename T>
__device__ __forceinline__ T uniform_load(const T *p, int64_t i) {
    T r;
    if constexpr (sizeof(T) % 8 == 0) {
        uint64_t w[sizeof(T) / 8];
        const const_u64_ptr q = (const_u64_ptr)(p + i);
#pragma unroll
        for (int j = 0; j < (int)(sizeof(T) / 8); ++j) w[j] = q[j];
        __builtin_memcpy(&r, w, sizeof(T));
    } else {
        static_assert(sizeof(T) == 4, "32-bit or multiple-of-64-bit elements");
        const uint32_t w = ((const __attribute__((address_space(4))) uint32_t *)(p + i))[0];
        __builtin_memcpy(&r, &w, sizeof(T));
    }
    return r;
}

struct Iso {
    float x, y, z, m0;
    double df;
    float om1, om2;  // 1 - exp(-dt/T), accurate for small dt/T
    float kap, ofs;  // 2 pi gamma_bar dt, 2 pi df dt
    double t1, t2;
    int cls;
};

__device__ __forceinline__ Iso load_iso(const AdjArgs &a, int64_t k, bool act) {
    Iso s;
    s.x = act ? a.x[k] : 0.f;
    s.y = act ? a.y[k] : 0.f;
    s.z = act ? a.z[k] : 0.f;
    s.m0 = act ? a.m0[k] : 0.f;
    const float df = act ? a.df[k] : 0.f;
    s.df = df;
    s.cls = act ? a.cls[k] : 0;
    s.t1 = act ? (double)a.t1c[s.cls] : 1.0;
    s.t2 = act ? (double)a.t2c[s.cls] : 1.0;
    s.om1 = (float)(-expm1(-a.dt / s.t1));
    s.om2 = (float)(-expm1(-a.dt / s.t2));
    s.kap = (float)(kTwoPi * kGammaBar * a.dt);
    s.ofs = (float)(kTwoPi * (double)df * a.dt);
    return s;
}

struct StepCoef {
    float wx, wy, wz, S, C, D3;
};

__device__ __forceinline__ StepCoef raster_coef(const AdjOp &op, const AdjArgs &a, const Iso &s, bool need_d3) {
    StepCoef r;
    float bx = op.b1r, by = op.b1i;
    if (op.param >= 0) {
        const float2 p = uniform_load(a.rfp, op.param);
        bx = p.x;
        by = p.y;
    }
    r.wx = -s.kap * bx;
    r.wy = -s.kap * by;
    r.wz = -(s.kap * (op.gx * s.x + op.gy * s.y + op.gz * s.z) + s.ofs);
    const float q = r.wx * r.wx + r.wy * r.wy + r.wz * r.wz;
    rot_coeffs(q, r.S, r.C, r.D3);
    (void)need_d3;
    return r;
}

// Rotation by -phi about z (the phase of Eq. 4, phi = 2 pi cyc), then
// decay over tau: cos phi = 1 - c1, sin phi = sn + sl (FP64 rounded to an
// FP32 pair), E2 = 1 - om2.
struct RelaxCoef {
    float c1, sn, sl, om2, om1;
};

__device__ __forceinline__ RelaxCoef relax_coef(const AdjOp &op, const Iso &s) {
    RelaxCoef r;
    const double cyc = op.cyc[0] * s.x + op.cyc[1] * s.y + op.cyc[2] * s.z + s.df * op.tau;
    double sh, ch;
    sincos(kPi * (cyc - rint(cyc)), &sh, &ch);  // half angle
    const double sn = 2.0 * sh * ch;
    r.sn = (float)sn;
    r.sl = (float)(sn - (double)r.sn);
    r.c1 = (float)(2.0 * sh * sh);
    r.om2 = (float)(-expm1(-op.tau / s.t2));
    r.om1 = (float)(-expm1(-op.tau / s.t1));
    return r;
}

// hi + lo <- hi + lo + d, exactly up to the rounding of d + lo.
__device__ __forceinline__ void acc_add(float &hi, float &lo, float d) {
    const float b = d + lo;
    const float t = hi + b;
    const float bb = t - hi;
    lo = (hi - (t - bb)) + (b - bb);
    hi = t;
}

// One op on the state (H, L); v receives the rotated state before relaxation
// (from H).
__device__ __forceinline__ void step(const AdjOp &op, const AdjArgs &a, const Iso &s, float *H, float *L, float *v) {
    float d[3];
    if (op.kind == 0) {
        const StepCoef c = raster_coef(op, a, s, false);
        const float ax = c.wy * H[2] - c.wz * H[1], ay = c.wz * H[0] - c.wx * H[2], az = c.wx * H[1] - c.wy * H[0];
        const float bx = c.wy * az - c.wz * ay, by = c.wz * ax - c.wx * az, bz = c.wx * ay - c.wy * ax;
        const float r[3] = {c.S * ax + c.C * bx, c.S * ay + c.C * by, c.S * az + c.C * bz};
#pragma unroll
        for (int i = 0; i < 3; ++i) v[i] = H[i] + r[i];
        d[0] = r[0] - s.om2 * v[0];
        d[1] = r[1] - s.om2 * v[1];
        d[2] = r[2] + s.om1 * (s.m0 - v[2]);
    } else {
        const RelaxCoef r = relax_coef(op, s);
        const float rx = (-r.c1 * H[0] + (r.sn * H[1] + r.sl * H[1])) + (-r.c1 * L[0] + r.sn * L[1]);
        const float ry = (-r.c1 * H[1] - (r.sn * H[0] + r.sl * H[0])) + (-r.c1 * L[1] - r.sn * L[0]);
        v[0] = H[0] + rx;
        v[1] = H[1] + ry;
        v[2] = H[2];
        d[0] = rx - r.om2 * v[0];
        d[1] = ry - r.om2 * v[1];
        d[2] = r.om1 * (s.m0 - (H[2] + L[2]));
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) acc_add(H[i], L[i], d[i]);
}

// --------------------------------------------------------------- forward
__global__ __launch_bounds__(kAdjWG) void k_adj_forward(AdjArgs a) {
    __shared__ float ws[kAdjWG / 64][2];
    const int64_t k = (int64_t)blockIdx.x * kAdjWG + threadIdx.x;
    const bool act = k < a.K;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const Iso s = load_iso(a, k, act);
    float H[3] = {0.f, 0.f, s.m0}, L[3] = {0.f, 0.f, 0.f}, v[3];
    for (int p = 0;; ++p) {
        if (p % a.every == 0 && p < a.n_ops && act) {
            float *c = a.ckpt + (int64_t)(p / a.every) * 3 * a.K + k;
            c[0] = H[0];
            c[a.K] = H[1];
            c[2 * a.K] = H[2];
        }
        const int q1 = uniform_load(a.sstart, p + 1);
        for (int q = uniform_load(a.sstart, p); q < q1; ++q) {  // samples at this boundary (Eq. 6)
            const float sx = wave_sum_lane63(H[0] + L[0]), sy = wave_sum_lane63(H[1] + L[1]);
            if (lane == 63) {
                ws[wave][0] = sx;
                ws[wave][1] = sy;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int w = 0; w < kAdjWG / 64; ++w) {
                    re += ws[w][0];
                    im += ws[w][1];
                }
                a.sig_part[(int64_t)blockIdx.x * a.N + uniform_load(a.sid, q)] = make_double2(re, im);
            }
            __syncthreads();
        }
        if (p == a.n_ops) break;
        step(load_op(a.ops, p), a, s, H, L, v);
    }
}

// -------------------------------------------------------------- backward
// lambda += the signal cotangent of the samples taken at boundary p.
__device__ __forceinline__ void add_cotangent(const AdjArgs &a, int p, float *LH, float *LL) {
    const int q1 = uniform_load(a.sstart, p + 1);
    for (int q = uniform_load(a.sstart, p); q < q1; ++q) {
        const double2 w = uniform_load(a.w, uniform_load(a.sid, q));
        const float wx = (float)w.x, wy = (float)w.y;
        acc_add(LH[0], LL[0], wx + (float)(w.x - (double)wx));
        acc_add(LH[1], LL[1], wy + (float)(w.y - (double)wy));
    }
}

struct TAcc {
    double r1, r2;  // raster steps: sum of lambda'_z (M'_z - M0), lambda'_xy . M'_xy
    double x1, x2;  // relaxation blocks: the same terms times tau
};

// Back through op `op` whose rotated state is v: lambda' = (LH, LL) on entry,
// lambda = (D R)^T lambda' on exit, formed as an increment and two-summed.
__device__ __forceinline__ void back_step(const AdjOp &op, const AdjArgs &a, const Iso &s, const float *v, float *LH,
                                          float *LL, TAcc &t, float2 *rfg, int lane) {
    float d[3];
    if (op.kind == 0) {
        const float Mx = v[0] - s.om2 * v[0], My = v[1] - s.om2 * v[1], Mz = v[2] + s.om1 * (s.m0 - v[2]);
        t.r2 += (double)(LH[0] * Mx + LH[1] * My);
        t.r1 += (double)(LH[2] * (Mz - s.m0));
        const float d1[3] = {-s.om2 * LH[0], -s.om2 * LH[1], -s.om1 * LH[2]};  // D lambda' - lambda'
        const float mu[3] = {LH[0] + d1[0], LH[1] + d1[1], LH[2] + d1[2]};
        const StepCoef c = raster_coef(op, a, s, true);
        if (op.param >= 0) {  // wave-uniform
            const float wv[3] = {v[1] * mu[2] - v[2] * mu[1], v[2] * mu[0] - v[0] * mu[2], v[0] * mu[1] - v[1] * mu[0]};
            const float ax = c.wy * wv[2] - c.wz * wv[1], ay = c.wz * wv[0] - c.wx * wv[2],
                        az = c.wx * wv[1] - c.wy * wv[0];
            const float bx = c.wy * az - c.wz * ay, by = c.wz * ax - c.wx * az;
            const float gx = -s.kap * (wv[0] - c.C * ax + c.D3 * bx);
            const float gy = -s.kap * (wv[1] - c.C * ay + c.D3 * by);
            const float sx = wave_sum_lane63(gx), sy = wave_sum_lane63(gy);
            if (lane == 63) {
                atomicAdd(&rfg[op.param].x, sx);
                atomicAdd(&rfg[op.param].y, sy);
            }
        }
        // R^T mu - mu = -S (w x mu) + C (w x (w x mu))
        const float ax = c.wy * mu[2] - c.wz * mu[1], ay = c.wz * mu[0] - c.wx * mu[2], az = c.wx * mu[1] - c.wy * mu[0];
        const float bx = c.wy * az - c.wz * ay, by = c.wz * ax - c.wx * az, bz = c.wx * ay - c.wy * ax;
        d[0] = d1[0] + (-c.S * ax + c.C * bx);
        d[1] = d1[1] + (-c.S * ay + c.C * by);
        d[2] = d1[2] + (-c.S * az + c.C * bz);
    } else {
        const RelaxCoef r = relax_coef(op, s);
        const float e2v0 = v[0] - r.om2 * v[0], e2v1 = v[1] - r.om2 * v[1];
        const float Mz = v[2] + r.om1 * (s.m0 - v[2]);
        t.x2 += (double)(LH[0] * e2v0 + LH[1] * e2v1) * op.tau;
        t.x1 += (double)(LH[2] * (Mz - s.m0)) * op.tau;
        // mu = E2 lambda'_xy; lambda_xy = P(phi) mu (the transpose of the forward's rotation by -phi)
        const float mx = LH[0] - r.om2 * LH[0], my = LH[1] - r.om2 * LH[1];
        const float rx = -r.c1 * mx - (r.sn * my + r.sl * my);
        const float ry = -r.c1 * my + (r.sn * mx + r.sl * mx);
        d[0] = (mx - LH[0]) + rx;
        d[1] = (my - LH[1]) + ry;
        d[2] = -r.om1 * LH[2];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) acc_add(LH[i], LL[i], d[i]);
}

// 4 waves per SIMD: 128 VGPRs.  LDS holds 25 KiB of accumulators per
// workgroup, so registers set the occupancy.
__global__ __launch_bounds__(kAdjWG) __attribute__((amdgpu_waves_per_eu(4))) void k_adj_backward(AdjArgs a) {
    __shared__ double tg[kAdjMaxClasses][2];
    __shared__ float2 rfg[kAdjMaxRf];
    const int64_t k = (int64_t)blockIdx.x * kAdjWG + threadIdx.x;
    const bool act = k < a.K;
    const int lane = threadIdx.x & 63, tid = threadIdx.x;
    for (int j = tid; j < a.n_rf; j += kAdjWG) rfg[j] = make_float2(0.f, 0.f);
    for (int j = tid; j < kAdjMaxClasses * 2; j += kAdjWG) tg[j >> 1][j & 1] = 0.0;
    __syncthreads();
    const Iso s = load_iso(a, k, act);
    float LH[3] = {0.f, 0.f, 0.f}, LL[3] = {0.f, 0.f, 0.f};
    TAcc t = {0.0, 0.0, 0.0, 0.0};
    add_cotangent(a, a.n_ops, LH, LL);
    const int n_seg = (a.n_ops + a.every - 1) / a.every;
    for (int seg = n_seg - 1; seg >= 0; --seg) {
        const int p0 = seg * a.every, p1 = min(p0 + a.every, a.n_ops);
        float H[3] = {0.f, 0.f, 0.f}, L[3] = {0.f, 0.f, 0.f}, v[3];
        if (act) {
            const float *c = a.ckpt + (int64_t)seg * 3 * a.K + k;
            H[0] = c[0];
            H[1] = c[a.K];
            H[2] = c[2 * a.K];
        }
        // sub-checkpoints in HBM, one column per thread (coalesced), so that
        // LDS holds only the gradient accumulators and occupancy is set by
        // registers
        for (int p = p0; p < p1; ++p) {
            if (act && ((p - p0) & (kAdjSub - 1)) == 0) {
                float *c = a.sub + (int64_t)((p - p0) / kAdjSub) * 3 * a.K + k;
                c[0] = H[0];
                c[a.K] = H[1];
                c[2 * a.K] = H[2];
            }
            step(load_op(a.ops, p), a, s, H, L, v);
        }
        const int n_sub = (p1 - p0 + kAdjSub - 1) / kAdjSub;
        for (int sb = n_sub - 1; sb >= 0; --sb) {
            const int q0 = p0 + sb * kAdjSub, cnt = min(kAdjSub, p1 - q0);
            float SL[3] = {0.f, 0.f, 0.f};
            if (act) {
                const float *c = a.sub + (int64_t)sb * 3 * a.K + k;
                H[0] = c[0];
                H[1] = c[a.K];
                H[2] = c[2 * a.K];
            }
            float V[kAdjSub][3];
#pragma unroll
            for (int i = 0; i < kAdjSub; ++i)
                if (i < cnt) step(load_op(a.ops, q0 + i), a, s, H, SL, V[i]);
#pragma unroll
            for (int i = kAdjSub - 1; i >= 0; --i) {
                if (i < cnt) {
                    back_step(load_op(a.ops, q0 + i), a, s, V[i], LH, LL, t, rfg, lane);
                    add_cotangent(a, q0 + i, LH, LL);
                }
            }
        }
    }
    if (act) {
        atomicAdd(&tg[s.cls][0], (t.r1 * a.dt + t.x1) / (s.t1 * s.t1));
        atomicAdd(&tg[s.cls][1], (t.r2 * a.dt + t.x2) / (s.t2 * s.t2));
    }
    __syncthreads();
    for (int j = tid; j < a.n_rf; j += kAdjWG) a.grf_part[(int64_t)blockIdx.x * a.n_rf + j] = rfg[j];
    for (int c = tid; c < a.n_classes; c += kAdjWG)
        a.gt_part[(int64_t)blockIdx.x * a.n_classes + c] = make_double2(tg[c][0], tg[c][1]);
}

// -------------------------------------------------------------- finalize
__global__ __launch_bounds__(256) void k_adj_sum_sig(const double2 *part, int grid, int N, double *sig) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    double re = 0.0, im = 0.0;
    for (int g = 0; g < grid; ++g) {
        const double2 p = part[(int64_t)g * N + n];
        re += p.x;
        im += p.y;
    }
    sig[2 * n] = re;
    sig[2 * n + 1] = im;
}

__global__ __launch_bounds__(256) void k_adj_sum_grad(const float2 *grf, const double2 *gt, int grid, int n_rf, int C,
                                                      float *grad_rf, double *g1, double *g2) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n_rf) {
        double re = 0.0, im = 0.0;
        for (int g = 0; g < grid; ++g) {
            const float2 p = grf[(int64_t)g * n_rf + j];
            re += p.x;
            im += p.y;
        }
        grad_rf[2 * j] = (float)re;
        grad_rf[2 * j + 1] = (float)im;
    }
    if (j < C) {
        double a = 0.0, b = 0.0;
        for (int g = 0; g < grid; ++g) {
            const double2 p = gt[(int64_t)g * C + j];
            a += p.x;
            b += p.y;
        }
        g1[j] = a;
        g2[j] = b;
    }
}

static int adj_grid(const AdjArgs &a) { return (int)((a.K + kAdjWG - 1) / kAdjWG); }

hipError_t launch_adj_forward(const AdjArgs &a, hipStream_t st) {
    if (a.K <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_forward, dim3(adj_grid(a)), dim3(kAdjWG), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_adj_backward(const AdjArgs &a, hipStream_t st) {
    if (a.K <= 0) return hipSuccess;
    if (a.n_rf > kAdjMaxRf || a.every > kAdjMaxEvery || a.every % kAdjSub || a.n_classes > kAdjMaxClasses)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adj_backward, dim3(adj_grid(a)), dim3(kAdjWG), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_adj_finalize(const AdjArgs &a, double *sig, float *grad_rf, double *grad_t1, double *grad_t2,
                               bool forward, hipStream_t st) {
    const int grid = adj_grid(a);
    if (forward) {
        if (a.N > 0)
            hipLaunchKernelGGL(k_adj_sum_sig, dim3((a.N + 255) / 256), dim3(256), 0, st, a.sig_part, grid, a.N, sig);
    } else {
        const int n = a.n_rf > a.n_classes ? a.n_rf : a.n_classes;
        hipLaunchKernelGGL(k_adj_sum_grad, dim3((n + 255) / 256), dim3(256), 0, st, a.grf_part, a.gt_part, grid,
                           a.n_rf, a.n_classes, grad_rf, grad_t1, grad_t2);
    }
    return hipGetLastError();
}

}  // namespace gbs

namespace gbs {

// Flags bad inputs of a gradient run: class index out of range, T1/T2 not > 0.
__global__ __launch_bounds__(256) void k_adj_validate(int64_t K, const int32_t *cls, int n_classes, const float *t1c,
                                                      const float *t2c, int *flag) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n_classes && !(t1c[k] > 0.f && t2c[k] > 0.f)) atomicOr(flag, 2);
    if (k < K && (cls[k] < 0 || cls[k] >= n_classes)) atomicOr(flag, 1);
}

hipError_t launch_adj_validate(int64_t K, const int32_t *cls, int n_classes, const float *t1c, const float *t2c,
                               int *flag, hipStream_t st) {
    const int64_t n = K > n_classes ? K : n_classes;
    hipLaunchKernelGGL(k_adj_validate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, K, cls, n_classes, t1c,
                       t2c, flag);
    return hipGetLastError();
}

}  // namespace gbs
