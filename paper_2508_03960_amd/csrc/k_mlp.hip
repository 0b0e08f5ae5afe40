// Learned RF-transition surrogate kernels for gfx950.
//
//  k_mlp_exact      exact transition T of the modelled RF subsequence (Eq. 7)
//                   for a batch of parameter tuples, FP64, one wavefront per
//                   tuple: the training data, the spot check and the exact
//                   fallback.
//  k_mlp_targets    T -> kResidualScale (K - K_ref): the frame (free
//                   precession of each half pulse removed), less the
//                   reference transition.
//  k_mlp_train_fb   forward and backward pass of one batch on
//                   v_mfma_f32_16x16x32_bf16, 16 samples per workgroup, one
//                   16-neuron tile per wavefront; tiles pass between layers
//                   through LDS in the B-operand order (see the k order below).
//  k_mlp_grad_adam  weight and bias gradients (contraction over the batch),
//                   then the Adam update of the FP32 master weights and the
//                   repacked BF16 MFMA fragments, one gradient tile per
//                   workgroup.
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
#include "rotation.hpp"

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

// Logistic function with the hardware reciprocal (v_rcp_f32, within 1 ulp):
// the IEEE-exact quotient costs nine VALU instructions per activation, a
// large share of the forward pass, for an error far below the BF16 weight
// rounding the network already carries.
__device__ __forceinline__ float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.f + __expf(-z)); }

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
    const double gdt = kTwoPi * kGammaBar * a.dt, k2 = gdt * gdt;
    Aff64 T = {{1, 0, 0, 0, 1, 0, 0, 0, 1}, {0, 0, 0}};
    for (int s = lo; s < hi; ++s) {
        const float4 w = a.wave[s];
        const double bx = s1 * w.x, by = s1 * w.y, bz = (double)w.z * z + boff;
        // Eq. A2 as R = (1 - cb |B|^2) I + ca [B]x + cb B B^T, with
        // ca = sin(theta) / |B| and cb = (1 - cos theta) / |B|^2 from their series
        const double B2 = fma(bx, bx, fma(by, by, bz * bz));
        double ca, cb;
        rot_coeffs(B2, gdt, k2, ca, cb);
        const double c0 = fma(-cb, B2, 1.0);
        const double qx = cb * bx, qy = cb * by, qz = cb * bz;
        const double pxy = qx * by, pxz = qx * bz, pyz = qy * bz;
        const double sx = ca * bx, sy = ca * by, sz = ca * bz;
        Aff64 U;
        U.a[0] = fma(qx, bx, c0);
        U.a[1] = pxy - sz;
        U.a[2] = pxz + sy;
        U.a[3] = pxy + sz;
        U.a[4] = fma(qy, by, c0);
        U.a[5] = pyz - sx;
        U.a[6] = pxz - sy;
        U.a[7] = pyz + sx;
        U.a[8] = fma(qz, bz, c0);
        U.b[0] = U.b[1] = U.b[2] = 0.0;
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
// One workgroup per 16 samples, kTrainWaves wavefronts: wavefront w computes
// neuron tile w (rows 16w..16w+15) of every 128-wide layer.  The next layer's
// B operand for chunk c is tiles 2c and 2c+1 at the same lane positions (see
// kperm), so each wavefront publishes its tile's BF16 (hi, lo) halves in LDS
// and reads the four chunks back after one barrier; the two exchange buffers
// alternate, so a write can only follow the barrier that ended the previous
// reads of its buffer.  The 12-output layer and the loss are computed by
// every wavefront (one tile, 8 MFMAs), which hands each of them dZ4 without
// another exchange; wavefront 0 alone stores them.
constexpr int kTrainWaves = 8;

struct TileHL {
    uint2 h, l;  // rows 4g..4g+3 of a tile, BF16 hi and lo halves
};

__device__ __forceinline__ uint2 pack4(const uint16_t *v) {
    return make_uint2((uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16));
}

__device__ __forceinline__ bf16x8 frag_of(uint2 a, uint2 b) {
    const uint4 u = make_uint4(a.x, a.y, b.x, b.y);
    bf16x8 r;
    __builtin_memcpy(&r, &u, 16);
    return r;
}

// B operands of the next layer from the exchange buffer.
__device__ __forceinline__ void frags_from_lds(const TileHL (*x)[64], int lane, bf16x8 *fh, bf16x8 *fl) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const TileHL t0 = x[2 * c][lane], t1 = x[2 * c + 1][lane];
        fh[c] = frag_of(t0.h, t1.h);
        fl[c] = frag_of(t0.l, t1.l);
    }
}

// Hidden-layer epilogue of one tile: z -> SiLU(z); keeps SiLU'(z) in sp for
// the backward pass and stores the activation (hi, lo) for the weight
// gradients.  row = first neuron of the lane (16w + 4g).
__device__ __forceinline__ TileHL hidden_tile(const f32x4 &acc, const MlpTrainArgs &a, int act_base, int row, int s,
                                              float *sp) {
    const int64_t B = a.B;
    uint16_t *ah = a.act_h + (act_base + row) * B + s;
    uint16_t *al = a.act_l + (act_base + row) * B + s;
    uint16_t hb[4], lb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float z = acc[r];
        const float sg = sigmoid(z);
        const float y = z * sg;
        sp[r] = sg * (1.f + z * (1.f - sg));
        hb[r] = bf16_bits(y);
        lb[r] = bf16_bits(y - bf16_float(hb[r]));
        ah[r * B] = hb[r];
        al[r * B] = lb[r];
    }
    return TileHL{pack4(hb), pack4(lb)};
}

// dZ = dH * SiLU'(Z) for one tile; stores dZ (hi, lo).
__device__ __forceinline__ TileHL backward_tile(const f32x4 &acc, const MlpTrainArgs &a, const float *sp, int dz_base,
                                                int row, int s) {
    const int64_t B = a.B;
    uint16_t *dh = a.dz_h + (dz_base + row) * B + s;
    uint16_t *dl = a.dz_l + (dz_base + row) * B + s;
    uint16_t hb[4], lb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float d = acc[r] * sp[r];
        hb[r] = bf16_bits(d);
        lb[r] = bf16_bits(d - bf16_float(hb[r]));
        dh[r * B] = hb[r];
        dl[r * B] = lb[r];
    }
    return TileHL{pack4(hb), pack4(lb)};
}

// acc += W(tile w) X over the four 32-neuron chunks, hi then lo per chunk.
__device__ __forceinline__ f32x4 dense_tile(f32x4 acc, const bf16x8 *A, const bf16x8 *fh, const bf16x8 *fl) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        acc = mfma(A[c], fh[c], acc);
        acc = mfma(A[c], fl[c], acc);
    }
    return acc;
}

__device__ __forceinline__ void load_a4(const uint4 *frags, int F, int lane, bf16x8 *A) {
#pragma unroll
    for (int c = 0; c < 4; ++c) A[c] = ld_frag(frags, F + c, lane);
}

__global__ __launch_bounds__(64 * kTrainWaves) void k_mlp_train_fb(MlpTrainArgs a) {
    __shared__ TileHL xch[2][kTrainWaves][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, col = lane & 15;
    const int row = 16 * w + 4 * g;  // first neuron of the lane's rows in tile w
    const int B = a.B;
    const int s = blockIdx.x * 16 + col;  // < B by the launch
    const int64_t j = (a.j0 + s) % a.N;
    const int64_t idx = (int64_t)(((uint64_t)a.pa * (uint64_t)j + a.pc) % (uint64_t)a.N);
    // Every global load of the pass is issued here: only the LDS exchanges
    // then separate the layers.
    float u[5], tgt[4];
    features(a.tuples + 5 * idx, a.norm, u);
    f32x4 b1, b2, b3, b4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = 4 * g + r;
        tgt[r] = o < 12 ? a.targets[12 * idx + o] : 0.f;
        b1[r] = a.params[kOffB1 + row + r];
        b2[r] = a.params[kOffB2 + row + r];
        b3[r] = a.params[kOffB3 + row + r];
        b4[r] = o < 12 ? a.params[kOffB4 + o] : 0.f;
    }
    const bf16x8 A1 = ld_frag(a.wf, kFragFwdL1 + w, lane), A4b = ld_frag(a.wb, kFragBwdL4 + w, lane);
    bf16x8 A2[4], A3[4], A4[4], A3b[4], A2b[4];
    load_a4(a.wf, kFragFwdL2 + 4 * w, lane, A2);
    load_a4(a.wf, kFragFwdL3 + 4 * w, lane, A3);
    load_a4(a.wf, kFragFwdL4, lane, A4);
    load_a4(a.wb, kFragBwdL3 + 4 * w, lane, A3b);
    load_a4(a.wb, kFragBwdL2 + 4 * w, lane, A2b);
    if (w == 0 && g == 0) {  // H0 rows: the 5 inputs, then zeros
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float v = r < 5 ? u[r < 5 ? r : 0] : 0.f;
            const uint16_t hb = bf16_bits(v);
            a.act_h[(int64_t)r * B + s] = hb;
            a.act_l[(int64_t)r * B + s] = bf16_bits(v - bf16_float(hb));
        }
    }
    bf16x8 fh[4], fl[4];
    f32x4 acc;
    float sp1[4], sp2[4], sp3[4];  // SiLU'(Z1..Z3) of the lane's rows
    // layer 1
    {
        bf16x8 xh, xl;
        input_frag(u, g, xh, xl);
        acc = mfma(A1, xh, b1);
        acc = mfma(A1, xl, acc);
        xch[0][w][lane] = hidden_tile(acc, a, 16, row, s, sp1);
    }
    // layers 2 and 3
    __syncthreads();
    frags_from_lds(xch[0], lane, fh, fl);
    acc = dense_tile(b2, A2, fh, fl);
    xch[1][w][lane] = hidden_tile(acc, a, 144, row, s, sp2);
    __syncthreads();
    frags_from_lds(xch[1], lane, fh, fl);
    acc = dense_tile(b3, A3, fh, fl);
    xch[0][w][lane] = hidden_tile(acc, a, 272, row, s, sp3);
    // layer 4 and the loss, in every wavefront
    __syncthreads();
    frags_from_lds(xch[0], lane, fh, fl);
    const f32x4 y = dense_tile(b4, A4, fh, fl);
    float dz[4], lsum = 0.f;
    const float scale = 2.f / (float)(B * 12);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = 4 * g + r;
        const float d = o < 12 ? y[r] - tgt[r] : 0.f;
        lsum += d * d;
        dz[r] = d * scale;
        if (w == 0) {
            const uint16_t hb = bf16_bits(dz[r]);
            a.dz_h[(int64_t)(384 + o) * B + s] = hb;
            a.dz_l[(int64_t)(384 + o) * B + s] = bf16_bits(dz[r] - bf16_float(hb));
        }
    }
    // dH3 = W4^T dZ4 (tile w), then dZ3
    {
        const float zero4[4] = {0.f, 0.f, 0.f, 0.f};
        bf16x8 dh, dl;
        make_frag(dz, zero4, dh, dl);
        acc = mfma(A4b, dh, f32x4{0.f, 0.f, 0.f, 0.f});
        acc = mfma(A4b, dl, acc);
    }
    xch[1][w][lane] = backward_tile(acc, a, sp3, 256, row, s);
    // dH2 = W3^T dZ3, then dZ2
    __syncthreads();
    frags_from_lds(xch[1], lane, fh, fl);
    acc = dense_tile(f32x4{0.f, 0.f, 0.f, 0.f}, A3b, fh, fl);
    xch[0][w][lane] = backward_tile(acc, a, sp2, 128, row, s);
    // dH1 = W2^T dZ2, then dZ1
    __syncthreads();
    frags_from_lds(xch[0], lane, fh, fl);
    acc = dense_tile(f32x4{0.f, 0.f, 0.f, 0.f}, A2b, fh, fl);
    backward_tile(acc, a, sp1, 0, row, s);
    if (w == 0) {
        lsum = wave_sum_lane63(lsum);
        if (lane == 63) atomicAdd(a.loss, lsum / (float)(B * 12));
    }
}

hipError_t launch_mlp_train_fb(const MlpTrainArgs &a, hipStream_t st) {
    if (a.B <= 0 || a.B % 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_train_fb, dim3((unsigned)(a.B / 16)), dim3(64 * kTrainWaves), 0, st, a);
    return hipGetLastError();
}

// ------------------------------------------------ packing, gradients, Adam
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

// ------------------------------------------------------- k_mlp_grad_adam
// Weight and bias gradients, 16 x 16 tiles: dW = dZ H^T, a contraction over
// the batch (D rows = output neurons, D columns = input neurons).  Layer 1
// has 8 x 2 tiles (weights over the 16 padded inputs, bias), layers 2 and 3
// 8 x 9 and layer 4 1 x 9; the ninth input tile of a layer is its bias,
// contracted against a ones column.  A workgroup takes one tile; its
// kGradWaves wavefronts split the batch's 32-sample chunks into contiguous
// ranges, their sums are added in wavefront order in LDS, and each of the
// 256 threads then owns one tile entry: it either writes the gradient or
// applies Adam to the parameter and repacks its BF16 fragments.
constexpr int kGradWaves = 8;
constexpr int kGradGroup = 4;

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) {
    const uint4 u = *(const uint4 *)p;
    bf16x8 r;
    __builtin_memcpy(&r, &u, 16);
    return r;
}

// Parameter index of entry (row, col) of gradient tile `tile`, -1 for padding.
__device__ __forceinline__ int param_of(int tile, int row, int col) {
    if (tile < 16) {
        const int o = 16 * (tile / 2) + row;
        if (tile & 1) return col == 0 ? kOffB1 + o : -1;
        return col < kMlpIn ? kOffW1 + kMlpIn * o + col : -1;
    }
    if (tile >= 160) {
        const int it = tile - 160;
        if (row >= kMlpOut) return -1;
        if (it == 8) return col == 0 ? kOffB4 + row : -1;
        return kOffW4 + kMlpH * row + 16 * it + col;
    }
    const bool l2 = tile < 88;
    const int t = tile - (l2 ? 16 : 88);
    const int o = 16 * (t / 9) + row, it = t % 9;
    if (it == 8) return col == 0 ? (l2 ? kOffB2 : kOffB3) + o : -1;
    return (l2 ? kOffW2 : kOffW3) + kMlpH * o + 16 * it + col;
}

__global__ __launch_bounds__(64 * kGradWaves) void k_mlp_grad_adam(MlpGradAdamArgs a) {
    __shared__ float part[kGradWaves][256];
    const int tile = blockIdx.x;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    int arow, brow, it;
    if (tile < 16) {
        it = tile % 2 == 1 ? 8 : 0;
        arow = 16 * (tile / 2);
        brow = 0;
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
    const int e = threadIdx.x;  // tile entry of the update (row e / 16, column e % 16)
    const int p = e < 256 ? param_of(tile, e / 16, e % 16) : -1;
    float m0 = 0.f, v0 = 0.f, w0 = 0.f;  // Adam state, loaded ahead of the contraction
    if (p >= 0 && !a.grad_out) {
        m0 = a.m[p];
        v0 = a.v[p];
        w0 = a.w[p];
    }
    const int nc = a.B / 32, c0 = q * nc / kGradWaves, c1 = (q + 1) * nc / kGradWaves;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    bf16x8 ones;
#pragma unroll
    for (int i = 0; i < 8; ++i) ones[i] = (__bf16)(col == 0 ? 1.f : 0.f);
    const uint16_t *pa_h = a.dz_h + (arow + col) * B + 8 * g, *pa_l = a.dz_l + (arow + col) * B + 8 * g;
    const uint16_t *pb_h = a.act_h + (brow + col) * B + 8 * g, *pb_l = a.act_l + (brow + col) * B + 8 * g;
    // chunks in groups of kGradGroup, every load of a group issued before its MFMAs
    int c = c0;
    for (; c < c1; c += kGradGroup) {
        const int n = c1 - c < kGradGroup ? c1 - c : kGradGroup;
        bf16x8 ah[kGradGroup], al[kGradGroup], bh[kGradGroup], bl[kGradGroup];
#pragma unroll
        for (int u = 0; u < kGradGroup; ++u) {
            if (u < n) {
                ah[u] = ld8(pa_h + 32 * (c + u));
                al[u] = ld8(pa_l + 32 * (c + u));
                if (!bias) {
                    bh[u] = ld8(pb_h + 32 * (c + u));
                    bl[u] = ld8(pb_l + 32 * (c + u));
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kGradGroup; ++u) {
            if (u < n) {
                if (bias) {
                    acc = mfma(ah[u], ones, acc);
                    acc = mfma(al[u], ones, acc);
                } else {
                    acc = mfma(ah[u], bh[u], acc);
                    acc = mfma(ah[u], bl[u], acc);
                    acc = mfma(al[u], bh[u], acc);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) part[q][(4 * g + r) * 16 + col] = acc[r];
    __syncthreads();
    if (p < 0) return;
    float gsum = 0.f;
#pragma unroll
    for (int k = 0; k < kGradWaves; ++k) gsum += part[k][e];
    if (a.grad_out) {
        a.grad_out[p] = gsum;
        return;
    }
    const float m = a.beta1 * m0 + (1.f - a.beta1) * gsum;
    const float v = a.beta2 * v0 + (1.f - a.beta2) * gsum * gsum;
    a.m[p] = m;
    a.v[p] = v;
    const float w = w0 - a.lr * (m * a.corr1) / (sqrtf(v * a.corr2) + a.eps);
    a.w[p] = w;
    const ParamPos pp = decode_param(p);
    if (!pp.bias) pack_weight(pp, bf16_bits(w), a.wf, a.wb);
}

hipError_t launch_mlp_grad_adam(const MlpGradAdamArgs &a, hipStream_t st) {
    if (a.B <= 0 || a.B % 32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_grad_adam, dim3(kGradTiles), dim3(64 * kGradWaves), 0, st, a);
    return hipGetLastError();
}

// Hidden-layer bias into the eight accumulator tiles (rows 16m + 4g + r).
__device__ __forceinline__ void bias_init(f32x4 *acc, const float *b, int g) {
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[m][r] = b[16 * m + 4 * g + r];
}

// B operands of the next layer: chunk c is D tiles 2c and 2c+1 (see kperm).
__device__ __forceinline__ void frags_from(const float (*h)[4], bf16x8 *fh, bf16x8 *fl) {
#pragma unroll
    for (int c = 0; c < 4; ++c) make_frag(h[2 * c], h[2 * c + 1], fh[c], fl[c]);
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
