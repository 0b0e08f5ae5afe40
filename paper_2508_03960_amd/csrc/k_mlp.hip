// Learned RF-transition surrogate kernels for gfx950.
//
//  k_mlp_exact      exact transition T of the modelled RF subsequence (Eq. 7)
//                   for a batch of parameter tuples, FP64, one wavefront per
//                   tuple: the training data, the spot check and the exact
//                   fallback.
//  k_mlp_targets    T -> kResidualScale (K - K_ref): the frame (free
//                   precession of each half pulse removed), less the
//                   reference transition.
//  k_mlp_train_fb   forward and backward pass of one batch, 16 samples per
//                   wavefront, on v_mfma_f32_16x16x32_bf16; activations stay
//                   in registers between layers (see the k order below).
//  k_mlp_wgrad      weight and bias gradients, split-K over the batch.
//  k_mlp_adam       Adam update of the FP32 master weights, then the BF16
//                   MFMA fragments are repacked.
//  k_mlp_infer      forward pass only, weights staged in LDS, 32 samples per
//                   wavefront and iteration, then K = K_ref + Y / scale and
//                   T = P(a) K P(a).
//
// MFMA 16x16x32 lane layout (lane l, g = l / 16): A holds row l % 16 and
// k = 8g..8g+7; B holds column l % 16 and the same k; D holds column l % 16
// and rows 4g..4g+3.  Layers are computed transposed, Y^T = W X^T, so D
// columns are samples and D rows are neurons.  A contraction may take its k
// in any order as long as both operands use the same one, so the k order of
// a 32-neuron chunk c is chosen to match what D already holds:
//     kperm(c, g, i) = 32c + (i < 4 ? 4g + i : 16 + 4g + i - 4)
// i.e. the B operand of the next layer is D tiles 2c and 2c+1 of this layer
// as they lie in the registers, and the weight fragments are packed in the
// same order.
#include "consts.hpp"
#include "device_math.hpp"
#include "mlp.hpp"

namespace gbs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ uint16_t bf16_bits(float v) {
    const __bf16 h = (__bf16)v;
    uint16_t u;
    __builtin_memcpy(&u, &h, 2);
    return u;
}

__device__ __forceinline__ float bf16_float(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }

// v = hi + lo with both in BF16 (round to nearest even).
__device__ __forceinline__ void split(float v, __bf16 &h, __bf16 &l) {
    h = (__bf16)v;
    l = (__bf16)(v - (float)h);
}

__device__ __forceinline__ bf16x8 ld_frag(const uint4 *frags, int F, int lane) {
    const uint4 u = frags[F * 64 + lane];
    bf16x8 r;
    __builtin_memcpy(&r, &u, 16);
    return r;
}

__device__ __forceinline__ void make_frag(const float *lo4, const float *hi4, bf16x8 &fh, bf16x8 &fl) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        __bf16 h, l;
        split(lo4[i], h, l);
        fh[i] = h;
        fl[i] = l;
        split(hi4[i], h, l);
        fh[4 + i] = h;
        fl[4 + i] = l;
    }
}

__device__ __forceinline__ float sigmoid(float z) { return 1.f / (1.f + __expf(-z)); }

__device__ __forceinline__ void features(const float *t, const MlpNorm &n, float u[5]) {
    const float v[5] = {t[0], t[1], __logf(t[2]), __logf(t[3]), t[4]};
#pragma unroll
    for (int k = 0; k < 5; ++k) u[k] = (v[k] - n.center[k]) * n.inv_scale[k];
}

// Layer-1 B operand: input feature kperm(0, g, i) -> 0..3 at g = 0, i < 4 and
// 4 at g = 1, i = 0; every other k is padding.
__device__ __forceinline__ void input_frag(const float u[5], int g, bf16x8 &fh, bf16x8 &fl) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float v = (g == 0 && i < 4) ? u[i & 3] : ((g == 1 && i == 0) ? u[4] : 0.f);
        __bf16 h, l;
        split(v, h, l);
        fh[i] = h;
        fl[i] = l;
    }
}

// ------------------------------------------------------------- k_mlp_exact
// One wavefront per tuple: lane l composes the contiguous chunk of steps
// [n l / 64, n (l + 1) / 64), then the 64 partial products are combined in a
// log2 tree through LDS (the later chunk on the left).
constexpr int kExactTuplesPerWG = 4;

struct Aff64 {
    double a[9], b[3];
};

// r = L o R (R first)
__device__ __forceinline__ void aff_mul(const Aff64 &L, const Aff64 &R, Aff64 &r) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r.a[3 * i + j] = L.a[3 * i] * R.a[j] + L.a[3 * i + 1] * R.a[3 + j] + L.a[3 * i + 2] * R.a[6 + j];
        r.b[i] = L.a[3 * i] * R.b[0] + L.a[3 * i + 1] * R.b[1] + L.a[3 * i + 2] * R.b[2] + L.b[i];
    }
}

__global__ __launch_bounds__(256) void k_mlp_exact(MlpExactArgs a) {
    __shared__ double lds[kExactTuplesPerWG][64][12];
    if (a.gate && *a.gate == 0) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * kExactTuplesPerWG + wave;
    const bool act = t < a.N;
    const int64_t src = act ? (a.idx ? (int64_t)a.idx[t] : t) : 0;
    const float *tp = a.tuples + 5 * src;
    const double z = act ? (double)tp[0] / (kGammaBar * a.g_ref) : 0.0;
    const double boff = act ? (double)tp[1] / kGammaBar : 0.0;
    const double e1 = act ? exp(-a.dt / (double)tp[2]) : 1.0, e2 = act ? exp(-a.dt / (double)tp[3]) : 1.0;
    const double s1 = act ? (double)tp[4] : 0.0;
    const int n = a.n_steps;
    const int lo = (int)(((int64_t)n * lane) >> 6), hi = (int)(((int64_t)n * (lane + 1)) >> 6);
    Aff64 T = {{1, 0, 0, 0, 1, 0, 0, 0, 1}, {0, 0, 0}};
    for (int s = lo; s < hi; ++s) {
        const float4 w = a.wave[s];
        const double bx = s1 * w.x, by = s1 * w.y, bz = (double)w.z * z + boff;
        const double nb = sqrt(bx * bx + by * by + bz * bz);
        Aff64 U = {{1, 0, 0, 0, 1, 0, 0, 0, 1}, {0, 0, 0}};
        if (nb > 0.0) {  // Eq. A2
            const double ux = bx / nb, uy = by / nb, uz = bz / nb;
            double sn, cs;
            sincos(-kTwoPi * kGammaBar * nb * a.dt, &sn, &cs);
            const double v = 1.0 - cs;
            U.a[0] = cs + ux * ux * v;
            U.a[1] = -uz * sn + ux * uy * v;
            U.a[2] = uy * sn + ux * uz * v;
            U.a[3] = uz * sn + ux * uy * v;
            U.a[4] = cs + uy * uy * v;
            U.a[5] = -ux * sn + uy * uz * v;
            U.a[6] = -uy * sn + ux * uz * v;
            U.a[7] = ux * sn + uy * uz * v;
            U.a[8] = cs + uz * uz * v;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {  // Eq. A1
            U.a[c] *= e2;
            U.a[3 + c] *= e2;
            U.a[6 + c] *= e1;
        }
        U.b[2] = 1.0 - e1;
        Aff64 Tn;
        aff_mul(U, T, Tn);
        T = Tn;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) lds[wave][lane][i] = T.a[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) lds[wave][lane][9 + i] = T.b[i];
    __syncthreads();
    for (int d = 1; d < 64; d <<= 1) {
        Aff64 L, R, r;
        const bool doit = (lane & (2 * d - 1)) == 0;
        if (doit) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                R.a[i] = lds[wave][lane][i];
                L.a[i] = lds[wave][lane + d][i];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                R.b[i] = lds[wave][lane][9 + i];
                L.b[i] = lds[wave][lane + d][9 + i];
            }
            aff_mul(L, R, r);
        }
        __syncthreads();
        if (doit) {
#pragma unroll
            for (int i = 0; i < 9; ++i) lds[wave][lane][i] = r.a[i];
#pragma unroll
            for (int i = 0; i < 3; ++i) lds[wave][lane][9 + i] = r.b[i];
        }
        __syncthreads();
    }
    if (act && lane < 12) a.out[12 * t + lane] = lds[wave][0][lane];
}

hipError_t launch_mlp_exact(const MlpExactArgs &a, hipStream_t st) {
    if (a.N <= 0) return hipSuccess;
    const int64_t wgs = (a.N + kExactTuplesPerWG - 1) / kExactTuplesPerWG;
    if (wgs > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_exact, dim3((unsigned)wgs), dim3(256), 0, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_f32(float *p, int64_t n, float v) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// z rotation P(alpha) of Eq. A2 (u = z): [[c, -s, 0], [s, c, 0], [0, 0, 1]].
// K = P(-a) A P(-a), k_b = P(-a) b  (inv = true), or the inverse map.
__device__ __forceinline__ void frame(const double *in, double c, double s, bool inv, double *out) {
    if (inv) s = -s;
    // P = [[c, -s, 0], [s, c, 0], [0, 0, 1]]
    double PA[9];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        PA[j] = c * in[j] - s * in[3 + j];
        PA[3 + j] = s * in[j] + c * in[3 + j];
        PA[6 + j] = in[6 + j];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        out[3 * i] = PA[3 * i] * c + PA[3 * i + 1] * s;
        out[3 * i + 1] = -PA[3 * i] * s + PA[3 * i + 1] * c;
        out[3 * i + 2] = PA[3 * i + 2];
    }
    out[9] = c * in[9] - s * in[10];
    out[10] = s * in[9] + c * in[10];
    out[11] = in[11];
}

__device__ __forceinline__ void frame_angle(const float *tp, double half, double &c, double &s) {
    double rev = -((double)tp[0] + (double)tp[1]) * half;
    rev -= rint(rev);
    sincos(kTwoPi * rev, &s, &c);
}

// Reference transition K_ref (frame coordinates, FP64) of tuple tp: the
// tabulated rotation interpolated at f = f_z + f_B0, its angle scaled by the
// B1 scale, relaxation over each half of the pulse on either side.
__device__ void ref_transition(const float *tp, const MlpNorm &n, double *k) {
    const double f = (double)tp[0] + (double)tp[1];
    double u = (f + kRefFmax) * ((kRefGrid - 1) / (2.0 * kRefFmax));
    u = u >= 0.0 ? (u <= kRefGrid - 1 ? u : (double)(kRefGrid - 1)) : 0.0;  // NaN -> 0
    int i0 = (int)u;
    i0 = i0 < kRefGrid - 2 ? i0 : kRefGrid - 2;
    const double w = u - i0;
    const float4 r0 = n.ref[i0], r1 = n.ref[i0 + 1];
    const double th = (1.0 - w) * r0.x + w * r1.x;
    double ax = (1.0 - w) * r0.y + w * r1.y, ay = (1.0 - w) * r0.z + w * r1.z, az = (1.0 - w) * r0.w + w * r1.w;
    const double nn = sqrt(ax * ax + ay * ay + az * az);
    if (nn > 0.0) {
        ax /= nn;
        ay /= nn;
        az /= nn;
    } else {
        ax = ay = 0.0;
        az = 1.0;
    }
    double sh, ch;
    sincos(0.5 * (double)tp[4] * th, &sh, &ch);
    const double qw = ch, qx = sh * ax, qy = sh * ay, qz = sh * az;
    const double R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw),     2 * (qx * qz + qy * qw),
                         2 * (qx * qy + qz * qw),     1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw),
                         2 * (qx * qz - qy * qw),     2 * (qy * qz + qx * qw),     1 - 2 * (qx * qx + qy * qy)};
    const double e1 = exp(-n.half / (double)tp[2]), e2 = exp(-n.half / (double)tp[3]);
    const double d[3] = {e2, e2, e1};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) k[3 * i + j] = d[i] * R[3 * i + j] * d[j];
        k[9 + i] = (1.0 - e1) * (d[i] * R[3 * i + 2] + (i == 2 ? 1.0 : 0.0));
    }
}

__global__ __launch_bounds__(256) void k_mlp_targets(const float *tuples, const double *T, int64_t N, MlpNorm norm,
                                                     float *K) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    double c, s, k[12], kr[12];
    frame_angle(tuples + 5 * t, norm.half, c, s);
    frame(T + 12 * t, c, s, true, k);
    ref_transition(tuples + 5 * t, norm, kr);
#pragma unroll
    for (int i = 0; i < 12; ++i) K[12 * t + i] = (float)(kResidualScale * (k[i] - kr[i]));
}

hipError_t launch_mlp_targets(const float *tuples, const double *T, int64_t N, const MlpNorm &norm, float *K,
                              hipStream_t st) {
    if (N <= 0) return hipSuccess;
    if (!norm.ref) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_targets, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, tuples, T, N, norm, K);
    return hipGetLastError();
}

// ---------------------------------------------------------- k_mlp_train_fb
// Hidden-layer epilogue: z -> SiLU(z); stores SiLU'(z) and the activation
// (hi, lo) for the weight gradients; leaves SiLU(z) in h.
__device__ __forceinline__ void hidden_out(const f32x4 *acc, float (*h)[4], const MlpTrainArgs &a,
                                           int sp_base, int act_base, int g, int s) {
    const int64_t B = a.B;
    // per-lane bases; the row offsets (16m + r) * B are wave-uniform
    float *sp = a.sp + (sp_base + 4 * g) * B + s;
    uint16_t *ah = a.act_h + (act_base + 4 * g) * B + s;
    uint16_t *al = a.act_l + (act_base + 4 * g) * B + s;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t off = (16 * m + r) * B;
            const float z = acc[m][r];
            const float sg = sigmoid(z);
            const float y = z * sg;
            h[m][r] = y;
            sp[off] = sg * (1.f + z * (1.f - sg));
            const uint16_t hb = bf16_bits(y);
            ah[off] = hb;
            al[off] = bf16_bits(y - bf16_float(hb));
        }
    }
}

__device__ __forceinline__ void frags_from(const float (*h)[4], bf16x8 *fh, bf16x8 *fl) {
#pragma unroll
    for (int c = 0; c < 4; ++c) make_frag(h[2 * c], h[2 * c + 1], fh[c], fl[c]);
}

__device__ __forceinline__ void bias_init(f32x4 *acc, const float *b, int g) {
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[m][r] = b[16 * m + 4 * g + r];
}

__device__ __forceinline__ void dense128(f32x4 *acc, const uint4 *wf, int fbase, const bf16x8 *fh,
                                        const bf16x8 *fl, int lane) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const bf16x8 A = ld_frag(wf, fbase + 4 * m + c, lane);
            acc[m] = mfma(A, fh[c], acc[m]);
            acc[m] = mfma(A, fl[c], acc[m]);
        }
        __builtin_amdgcn_sched_barrier(0);  // keeps fragment loads from piling up in registers
    }
}

// dZ = dH * SiLU'(Z); stores dZ (hi, lo); leaves dZ in h.
__device__ __forceinline__ void backward_out(const f32x4 *acc, float (*h)[4], const MlpTrainArgs &a,
                                             int sp_base, int dz_base, int g, int s) {
    const int64_t B = a.B;
    const float *sp = a.sp + (sp_base + 4 * g) * B + s;
    uint16_t *dh = a.dz_h + (dz_base + 4 * g) * B + s;
    uint16_t *dl = a.dz_l + (dz_base + 4 * g) * B + s;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t off = (16 * m + r) * B;
            const float d = acc[m][r] * sp[off];
            h[m][r] = d;
            const uint16_t hb = bf16_bits(d);
            dh[off] = hb;
            dl[off] = bf16_bits(d - bf16_float(hb));
        }
    }
}

__global__ __launch_bounds__(64) void k_mlp_train_fb(MlpTrainArgs a) {
    const int lane = threadIdx.x;
    const int g = lane >> 4, col = lane & 15;
    const int B = a.B;
    const int s = blockIdx.x * 16 + col;  // < B by the launch
    const int64_t j = (a.j0 + s) % a.N;
    const int64_t idx = (int64_t)(((uint64_t)a.pa * (uint64_t)j + a.pc) % (uint64_t)a.N);
    float u[5];
    features(a.tuples + 5 * idx, a.norm, u);
    if (g == 0) {  // H0 rows: the 5 inputs, then zeros
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float v = r < 5 ? u[r < 5 ? r : 0] : 0.f;
            const uint16_t hb = bf16_bits(v);
            a.act_h[(int64_t)r * B + s] = hb;
            a.act_l[(int64_t)r * B + s] = bf16_bits(v - bf16_float(hb));
        }
    }
    f32x4 acc[8];
    float h[8][4];
    bf16x8 fh[4], fl[4];
    // layer 1
    {
        bf16x8 xh, xl;
        input_frag(u, g, xh, xl);
        bias_init(acc, a.params + kOffB1, g);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const bf16x8 A = ld_frag(a.wf, kFragFwdL1 + m, lane);
            acc[m] = mfma(A, xh, acc[m]);
            acc[m] = mfma(A, xl, acc[m]);
        }
        hidden_out(acc, h, a, 0, 16, g, s);
    }
    // layers 2 and 3
    frags_from(h, fh, fl);
    bias_init(acc, a.params + kOffB2, g);
    dense128(acc, a.wf, kFragFwdL2, fh, fl, lane);
    hidden_out(acc, h, a, 128, 144, g, s);
    frags_from(h, fh, fl);
    bias_init(acc, a.params + kOffB3, g);
    dense128(acc, a.wf, kFragFwdL3, fh, fl, lane);
    hidden_out(acc, h, a, 256, 272, g, s);
    // layer 4 and the loss
    frags_from(h, fh, fl);
    f32x4 y;
#pragma unroll
    for (int r = 0; r < 4; ++r) y[r] = (4 * g + r < 12) ? a.params[kOffB4 + ((4 * g + r) % 12)] : 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const bf16x8 A = ld_frag(a.wf, kFragFwdL4 + c, lane);
        y = mfma(A, fh[c], y);
        y = mfma(A, fl[c], y);
    }
    float dz[4], lsum = 0.f;
    const float scale = 2.f / (float)(B * 12);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = 4 * g + r;
        float d = 0.f;
        if (o < 12) d = y[r] - a.targets[12 * idx + o];
        lsum += d * d;
        dz[r] = d * scale;
        const uint16_t hb = bf16_bits(dz[r]);
        a.dz_h[(int64_t)(384 + o) * B + s] = hb;
        a.dz_l[(int64_t)(384 + o) * B + s] = bf16_bits(dz[r] - bf16_float(hb));
    }
    // dH3 = W4^T dZ4
    {
        const float zero4[4] = {0.f, 0.f, 0.f, 0.f};
        bf16x8 dh, dl;
        make_frag(dz, zero4, dh, dl);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const bf16x8 A = ld_frag(a.wb, kFragBwdL4 + m, lane);
            acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
            acc[m] = mfma(A, dh, acc[m]);
            acc[m] = mfma(A, dl, acc[m]);
        }
    }
    backward_out(acc, h, a, 256, 256, g, s);  // dZ3
    frags_from(h, fh, fl);
#pragma unroll
    for (int m = 0; m < 8; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
    dense128(acc, a.wb, kFragBwdL3, fh, fl, lane);  // dH2 = W3^T dZ3
    backward_out(acc, h, a, 128, 128, g, s);        // dZ2
    frags_from(h, fh, fl);
#pragma unroll
    for (int m = 0; m < 8; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
    dense128(acc, a.wb, kFragBwdL2, fh, fl, lane);  // dH1 = W2^T dZ2
    backward_out(acc, h, a, 0, 0, g, s);            // dZ1
    lsum = wave_sum_lane63(lsum);
    if (lane == 63) atomicAdd(a.loss, lsum / (float)(B * 12));
}

hipError_t launch_mlp_train_fb(const MlpTrainArgs &a, hipStream_t st) {
    if (a.B <= 0 || a.B % 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_train_fb, dim3((unsigned)(a.B / 16)), dim3(64), 0, st, a);  // 16 samples per wavefront
    return hipGetLastError();
}

// -------------------------------------------------------------- k_mlp_wgrad
__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) {
    const uint4 u = *(const uint4 *)p;
    bf16x8 r;
    __builtin_memcpy(&r, &u, 16);
    return r;
}

__global__ __launch_bounds__(64) void k_mlp_wgrad(MlpGradArgs a) {
    const int tile = blockIdx.x, sl = blockIdx.y;
    const int lane = threadIdx.x, g = lane >> 4, col = lane & 15;
    int arow, brow, it;
    if (tile < 16) {
        it = tile % 2;
        arow = 16 * (tile / 2);
        brow = 0;
        it = it == 1 ? 8 : 0;
    } else if (tile < 88) {
        const int t = tile - 16;
        it = t % 9;
        arow = 128 + 16 * (t / 9);
        brow = 16 + 16 * it;
    } else if (tile < 160) {
        const int t = tile - 88;
        it = t % 9;
        arow = 256 + 16 * (t / 9);
        brow = 144 + 16 * it;
    } else {
        it = tile - 160;
        arow = 384;
        brow = 272 + 16 * it;
    }
    const bool bias = it == 8;
    const int64_t B = a.B;
    const int s0 = sl * a.slice;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    bf16x8 ones;
#pragma unroll
    for (int i = 0; i < 8; ++i) ones[i] = (__bf16)(col == 0 ? 1.f : 0.f);
    for (int k = 0; k < a.slice; k += 32) {
        const int64_t oa = (arow + col) * B + s0 + k + 8 * g;
        const bf16x8 ah = ld8(a.dz_h + oa), al = ld8(a.dz_l + oa);
        if (bias) {
            acc = mfma(ah, ones, acc);
            acc = mfma(al, ones, acc);
        } else {
            const int64_t ob = (brow + col) * B + s0 + k + 8 * g;
            const bf16x8 bh = ld8(a.act_h + ob), bl = ld8(a.act_l + ob);
            acc = mfma(ah, bh, acc);
            acc = mfma(ah, bl, acc);
            acc = mfma(al, bh, acc);
        }
    }
    float *o = a.part + ((int64_t)sl * kGradTiles + tile) * 256;
#pragma unroll
    for (int r = 0; r < 4; ++r) o[(4 * g + r) * 16 + col] = acc[r];
}

hipError_t launch_mlp_wgrad(const MlpGradArgs &a, hipStream_t st) {
    if (a.B <= 0 || a.slice <= 0 || a.slice % 32 || a.B % a.slice) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(kGradTiles, a.B / a.slice), dim3(64), 0, st, a);
    return hipGetLastError();
}

// --------------------------------------------------------- packing, Adam
struct ParamPos {
    int layer;  // 1..4
    bool bias;
    int o, i;
};

__device__ __forceinline__ ParamPos decode_param(int p) {
    ParamPos q{};
    if (p < kOffB1) q = {1, false, p / 5, p % 5};
    else if (p < kOffW2) q = {1, true, p - kOffB1, 0};
    else if (p < kOffB2) q = {2, false, (p - kOffW2) / 128, (p - kOffW2) % 128};
    else if (p < kOffW3) q = {2, true, p - kOffB2, 0};
    else if (p < kOffB3) q = {3, false, (p - kOffW3) / 128, (p - kOffW3) % 128};
    else if (p < kOffW4) q = {3, true, p - kOffB3, 0};
    else if (p < kOffB4) q = {4, false, (p - kOffW4) / 128, (p - kOffW4) % 128};
    else q = {4, true, p - kOffB4, 0};
    return q;
}

// Gradient tile, row and column of a parameter (see k_mlp_wgrad).
__device__ __forceinline__ void grad_pos(const ParamPos &q, int &tile, int &row, int &col) {
    const int it = q.bias ? 8 : q.i / 16;
    col = q.bias ? 0 : q.i % 16;
    row = q.o % 16;
    if (q.layer == 1) tile = (q.o / 16) * 2 + (q.bias ? 1 : 0);
    else if (q.layer == 2) tile = 16 + (q.o / 16) * 9 + it;
    else if (q.layer == 3) tile = 88 + (q.o / 16) * 9 + it;
    else tile = 160 + it;
}

// Inverse of kperm within a 32-chunk: k % 32 -> (g, i).
__device__ __forceinline__ void kperm_inv(int q, int &g, int &i) {
    const int half = q >> 4, qq = q & 15;
    g = qq >> 2;
    i = (qq & 3) + 4 * half;
}

__device__ __forceinline__ void pack_weight(const ParamPos &q, uint16_t v, uint16_t *wf, uint16_t *wb) {
    // forward: rows = o, k = i
    {
        int g, i;
        kperm_inv(q.i % 32, g, i);
        const int c = q.i / 32, m = q.o / 16;
        const int F = q.layer == 1 ? kFragFwdL1 + m
                    : q.layer == 2 ? kFragFwdL2 + 4 * m + c
                    : q.layer == 3 ? kFragFwdL3 + 4 * m + c
                                   : kFragFwdL4 + c;
        wf[(F * 64 + 16 * g + (q.o % 16)) * 8 + i] = v;
    }
    if (q.layer >= 2) {  // backward: rows = i, k = o
        int g, i;
        kperm_inv(q.o % 32, g, i);
        const int c = q.o / 32, m = q.i / 16;
        const int F = q.layer == 2 ? kFragBwdL2 + 4 * m + c
                    : q.layer == 3 ? kFragBwdL3 + 4 * m + c
                                   : kFragBwdL4 + m;
        wb[(F * 64 + 16 * g + (q.i % 16)) * 8 + i] = v;
    }
}

__global__ __launch_bounds__(256) void k_mlp_pack(const float *w, uint16_t *wf, uint16_t *wb) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kMlpParams) return;
    const ParamPos q = decode_param(p);
    if (!q.bias) pack_weight(q, bf16_bits(w[p]), wf, wb);
}

hipError_t launch_mlp_pack(const float *w, uint16_t *wf, uint16_t *wb, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_pack, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, w, wf, wb);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_mlp_adam(MlpAdamArgs a) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kMlpParams) return;
    const ParamPos q = decode_param(p);
    int tile, row, col;
    grad_pos(q, tile, row, col);
    float gsum = 0.f;
    for (int sl = 0; sl < a.n_slices; ++sl) gsum += a.part[((int64_t)sl * kGradTiles + tile) * 256 + row * 16 + col];
    if (a.grad_out) {
        a.grad_out[p] = gsum;
        return;
    }
    const float m = a.beta1 * a.m[p] + (1.f - a.beta1) * gsum;
    const float v = a.beta2 * a.v[p] + (1.f - a.beta2) * gsum * gsum;
    a.m[p] = m;
    a.v[p] = v;
    const float w = a.w[p] - a.lr * (m * a.corr1) / (sqrtf(v * a.corr2) + a.eps);
    a.w[p] = w;
    if (!q.bias) pack_weight(q, bf16_bits(w), a.wf, a.wb);
}

hipError_t launch_mlp_adam(const MlpAdamArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

// -------------------------------------------------------------- k_mlp_infer
constexpr int kInferWG = 512;  // 8 wavefronts share one LDS copy of the weights

// Tuple s of an inference launch (s < N).
__device__ __forceinline__ void infer_tuple(const MlpInferArgs &a, int64_t s, float tp[5]) {
    if (a.src_z) {
        tp[0] = (float)(a.fz_per_m * (double)a.src_z[s]);
        tp[1] = a.src_df[s];
        tp[2] = a.src_t1[s];
        tp[3] = a.src_t2[s];
        tp[4] = 1.f;
    } else {
        const float *p = a.tuples + 5 * (a.idx ? (int64_t)a.idx[s] : s);
#pragma unroll
        for (int i = 0; i < 5; ++i) tp[i] = p[i];
    }
}

__global__ __launch_bounds__(kInferWG) void k_mlp_infer(MlpInferArgs a) {
    __shared__ uint4 sw[kFragFwd * 64];
    __shared__ float sk[kInferWG / 64][32][12];
    for (int i = threadIdx.x; i < kFragFwd * 64; i += kInferWG) sw[i] = a.wf[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    const int64_t n_tiles = (a.N + 31) / 32;
    constexpr int kWaves = kInferWG / 64;
    for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < n_tiles; tile += (int64_t)gridDim.x * kWaves) {
        f32x4 acc[2][8];
        bf16x8 fh[2][4], fl[2][4];
        // layer 1
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int64_t s = tile * 32 + nt * 16 + col;
            float u[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            if (s < a.N) {
                float tp[5];
                infer_tuple(a, s, tp);
                features(tp, a.norm, u);
            }
            input_frag(u, g, fh[nt][0], fl[nt][0]);
            bias_init(acc[nt], a.params + kOffB1, g);
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const bf16x8 A = ld_frag(sw, kFragFwdL1 + m, lane);
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                acc[nt][m] = mfma(A, fh[nt][0], acc[nt][m]);
                acc[nt][m] = mfma(A, fl[nt][0], acc[nt][m]);
            }
        }
        // layers 2, 3
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                float h[8][4];
#pragma unroll
                for (int m = 0; m < 8; ++m)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float z = acc[nt][m][r];
                        h[m][r] = z * sigmoid(z);
                    }
                frags_from(h, fh[nt], fl[nt]);
                bias_init(acc[nt], a.params + (layer == 0 ? kOffB2 : kOffB3), g);
            }
            const int fb = layer == 0 ? kFragFwdL2 : kFragFwdL3;
#pragma unroll
            for (int m = 0; m < 8; ++m)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const bf16x8 A = ld_frag(sw, fb + 4 * m + c, lane);
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt) {
                        acc[nt][m] = mfma(A, fh[nt][c], acc[nt][m]);
                        acc[nt][m] = mfma(A, fl[nt][c], acc[nt][m]);
                    }
                }
        }
        // layer 4
        f32x4 y[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            float h[8][4];
#pragma unroll
            for (int m = 0; m < 8; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float z = acc[nt][m][r];
                    h[m][r] = z * sigmoid(z);
                }
            frags_from(h, fh[nt], fl[nt]);
#pragma unroll
            for (int r = 0; r < 4; ++r) y[nt][r] = (4 * g + r < 12) ? a.params[kOffB4 + ((4 * g + r) % 12)] : 0.f;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const bf16x8 A = ld_frag(sw, kFragFwdL4 + c, lane);
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                y[nt] = mfma(A, fh[nt][c], y[nt]);
                y[nt] = mfma(A, fl[nt][c], y[nt]);
            }
        }
        // gather the 12 outputs of each sample in one lane, then T = P(a) K P(a)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (4 * g + r < 12) sk[wave][nt * 16 + col][4 * g + r] = y[nt][r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int64_t s = tile * 32 + lane;
        if (lane < 32 && s < a.N) {
            double k[12], T[12], c, sn;
            float tp[5];
            infer_tuple(a, s, tp);
            ref_transition(tp, a.norm, k);
#pragma unroll
            for (int i = 0; i < 12; ++i) k[i] += (double)sk[wave][lane][i] * (1.0 / kResidualScale);
            frame_angle(tp, a.norm.half, c, sn);
            frame(k, c, sn, false, T);
            if (a.rows) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    a.rows[i * a.row_stride + s] =
                        make_float4((float)T[3 * i], (float)T[3 * i + 1], (float)T[3 * i + 2], (float)T[9 + i]);
            } else {
                float *o = a.out + 12 * s;
#pragma unroll
                for (int i = 0; i < 12; ++i) o[i] = (float)T[i];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

hipError_t launch_mlp_infer(const MlpInferArgs &a, hipStream_t st) {
    if (a.N <= 0) return hipSuccess;
    if (!a.norm.ref || (!a.rows && !a.out) || (!a.src_z && !a.tuples)) return hipErrorInvalidValue;
    const int64_t tiles = (a.N + 31) / 32;
    const int64_t wgs = (tiles + kInferWG / 64 - 1) / (kInferWG / 64);
    const unsigned grid = (unsigned)(wgs < 256 ? wgs : 256);  // one resident workgroup per CU
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(kInferWG), 0, st, a);
    return hipGetLastError();
}

// ------------------------------------------------- use inside a simulation
// Tuples of the z-group table rows (coord, T1, T2, df) for B1 scale 1.
__global__ __launch_bounds__(256) void k_surr_tuples(const float4 *gtab, int64_t n, double fz_per_m,
                                                     float *tuples) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float4 r = gtab[t];
    float *o = tuples + 5 * t;
    o[0] = (float)(fz_per_m * (double)r.x);
    o[1] = r.w;
    o[2] = r.y;
    o[3] = r.z;
    o[4] = 1.f;
}

hipError_t launch_surr_tuples(const float4 *gtab, int64_t n, double fz_per_m, float *tuples, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_surr_tuples, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gtab, n, fz_per_m,
                       tuples);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_surr_store(const float *T32, int64_t n, double *T64) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 12 * n) T64[t] = T32[t];
}

hipError_t launch_surr_store(const float *T32, int64_t n, double *T64, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_surr_store, dim3((unsigned)((12 * n + 255) / 256)), dim3(256), 0, st, T32, n, T64);
    return hipGetLastError();
}

// Tuples of phantom isochromats idx[0 .. n) for B1 scale 1:
// (fz_per_m z, df, t1, t2, 1).
__global__ __launch_bounds__(256) void k_surr_iso_tuples(const float *z, const float *df, const float *t1,
                                                         const float *t2, const int32_t *idx, int n, double fz_per_m,
                                                         float *tuples) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t k = idx[t];
    float *o = tuples + 5 * (int64_t)t;
    o[0] = (float)(fz_per_m * (double)z[k]);
    o[1] = df[k];
    o[2] = t1[k];
    o[3] = t2[k];
    o[4] = 1.f;
}

hipError_t launch_surr_iso_tuples(const float *z, const float *df, const float *t1, const float *t2,
                                  const int32_t *idx, int n, double fz_per_m, float *tuples, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_surr_iso_tuples, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, z, df, t1, t2, idx, n,
                       fz_per_m, tuples);
    return hipGetLastError();
}

// Entry c of network transition k: T32[12 idx[k] + c], or from the row planes
// (rows[i * stride + idx[k]] = (A_i0, A_i1, A_i2, b_i)).
__device__ __forceinline__ float checked_entry(const float *T32, const float4 *rows, int64_t stride, int64_t k,
                                               int c) {
    if (!rows) return T32[12 * k + c];
    const int i = c < 9 ? c / 3 : c - 9, j = c < 9 ? c % 3 : 3;
    const float4 r = rows[i * stride + k];
    return j == 0 ? r.x : j == 1 ? r.y : j == 2 ? r.z : r.w;
}

// max |T_mlp - T_exact| over the checked transitions; sets *fallback when it
// exceeds tol (or is NaN).  One workgroup.
__global__ __launch_bounds__(256) void k_surr_check(const float *T32, const float4 *rows, int64_t stride,
                                                    const int32_t *idx, const double *exact, int n_check, float tol,
                                                    float *residual, int32_t *fallback) {
    __shared__ float red[256];
    float mx = 0.f;
    for (int e = threadIdx.x; e < 12 * n_check; e += 256) {
        const int k = e / 12, c = e % 12;
        const float d = fabsf((float)(exact[e] - (double)checked_entry(T32, rows, stride, idx[k], c)));
        mx = (d > mx || d != d) ? d : mx;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const float o = red[threadIdx.x + w];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float r = red[0];
        *residual = r;
        *fallback = (r > tol || r != r) ? 1 : 0;
    }
}

hipError_t launch_surr_check(const float *T32, const int32_t *idx, const double *exact, int n_check, float tol,
                             float *residual, int32_t *fallback, hipStream_t st) {
    hipLaunchKernelGGL(k_surr_check, dim3(1), dim3(256), 0, st, T32, (const float4 *)nullptr, (int64_t)0, idx, exact,
                       n_check, tol, residual, fallback);
    return hipGetLastError();
}

hipError_t launch_surr_check_rows(const float4 *rows, int64_t stride, const int32_t *idx, const double *exact,
                                  int n_check, float tol, float *residual, int32_t *fallback, hipStream_t st) {
    hipLaunchKernelGGL(k_surr_check, dim3(1), dim3(256), 0, st, (const float *)nullptr, rows, stride, idx, exact,
                       n_check, tol, residual, fallback);
    return hipGetLastError();
}

}  // namespace gbs
