// Grouped-isochromat kernels for gfx950 (Sec. 2.3, 2.4).
//
//  k_compose   combined transition T = U_{N-1} ... U_0 (Eq. 7) once per group,
//              FP64.  One wavefront per group: each lane composes a contiguous
//              chunk of steps, then the 64 partial products are combined in a
//              log2 tree through LDS (later chunk on the left).
//  k_fold      per operation, T' = T o P with the tissue part and the
//              own-axis phase of the preceding B1 = 0 map P (Eq. 4, 5), FP64,
//              rounded once to FP32.
//  k_tables    per-group factors of the remaining B1 = 0 map parts.
//  k_sweep     one coalesced sweep over the group-sorted isochromats that
//              applies a run of grouped operations with the state in
//              registers: pre-map phases, group transitions, and the group
//              sums of each with-ADC subsequence (Eq. 9) reduced across the
//              wavefront (one group per wavefront in the common case), then
//              FP64 atomics.
//  k_adc_eval  every ADC sample from the group sums (Eq. 8 with Eq. 10), FP64
//              phase reduced modulo one turn, FP64 accumulation.
//  k_init_state, k_gather_state4, k_gather_state4x4, k_gather_state
//              the state into the group-sorted layout (when the first sweep
//              does not start it from (0, 0, M0) itself) and back into the
//              caller's order (from the last sweep's 16-byte rows, or from the
//              per-component arrays after plain stepping).
#include "device_math.hpp"
#include "kernels.hpp"
#include "rotation.hpp"

namespace gbs {

// ---------------------------------------------------------------- k_compose
constexpr int kComposeGroupsPerWG = 4;
typedef const __attribute__((address_space(1))) float *compose_gf32;

struct Aff {
    double a[9];  // row-major 3x3
    double b[3];
};

__device__ __forceinline__ void aff_identity(Aff &t) {
#pragma unroll
    for (int i = 0; i < 9; ++i) t.a[i] = (i % 4 == 0) ? 1.0 : 0.0;
    t.b[0] = t.b[1] = t.b[2] = 0.0;
}

// r = L o R (apply R first, then L)
__device__ __forceinline__ void aff_compose(const Aff &L, const Aff &R, Aff &r) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r.a[3 * i + j] = L.a[3 * i] * R.a[j] + L.a[3 * i + 1] * R.a[3 + j] + L.a[3 * i + 2] * R.a[6 + j];
        r.b[i] = L.a[3 * i] * R.b[0] + L.a[3 * i + 1] * R.b[1] + L.a[3 * i + 2] * R.b[2] + L.b[i];
    }
}

__global__ __launch_bounds__(256) void k_compose(const RfJobDev *__restrict__ jobs, double dt) {
    __shared__ double lds[kComposeGroupsPerWG][64][12];
    const RfJobDev j = jobs[blockIdx.y];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * kComposeGroupsPerWG + wave;
    const bool act = g < j.n_groups;
    float4 p = act ? j.gtab[g] : make_float4(0.f, __builtin_inff(), __builtin_inff(), 0.f);
    const double coord = p.x, t1 = p.y, t2 = p.z;
    const double boff = (double)p.w / kGammaBar;
    const double e1 = exp(-dt / t1), e2 = exp(-dt / t2);
    const double gdt = kTwoPi * kGammaBar * dt, k2 = gdt * gdt;
    const int n = j.n_steps;
    const int lo = (int)(((int64_t)n * lane) >> 6), hi = (int)(((int64_t)n * (lane + 1)) >> 6);
    // (B1 re, B1 im, gradient on the job's axis) of step s, through the
    // global address space, the index clamped into the waveform
    const int gcol = 3 + j.axis;  // gx, gy, gz follow b1r, b1i, b1sq in StepW
    auto step_in = [&](int s) {
        const compose_gf32 w = (compose_gf32)(j.wave + min(s, n - 1));
        return make_float3(w[0], w[1], w[gcol]);
    };
    // U = D R (Eq. A1, Eq. A2) with R = (1 - cb |B|^2) I + ca [B]x + cb B B^T,
    // ca = sin(theta) / |B| and cb = (1 - cos theta) / |B|^2 from their series
    // (no square root or division; B = 0 gives the identity)
    auto step_u = [&](const float3 &w, Aff &U) {
        const double bx = w.x, by = w.y, bz = (double)w.z * coord + boff;
        const double B2 = fma(bx, bx, fma(by, by, bz * bz));
        double ca, cb;
        rot_coeffs(B2, gdt, k2, ca, cb);
        const double c0 = fma(-cb, B2, 1.0);
        const double qx = cb * bx, qy = cb * by, qz = cb * bz;
        const double pxy = qx * by, pxz = qx * bz, pyz = qy * bz;
        const double sx = ca * bx, sy = ca * by, sz = ca * bz;
        U.a[0] = fma(qx, bx, c0) * e2;
        U.a[1] = (pxy - sz) * e2;
        U.a[2] = (pxz + sy) * e2;
        U.a[3] = (pxy + sz) * e2;
        U.a[4] = fma(qy, by, c0) * e2;
        U.a[5] = (pyz - sx) * e2;
        U.a[6] = (pxz - sy) * e1;
        U.a[7] = (pyz + sx) * e1;
        U.a[8] = fma(qz, bz, c0) * e1;
        U.b[0] = U.b[1] = 0.0;
        U.b[2] = 1.0 - e1;
    };
    // The lane's steps in fours: each of w0..w3 is consumed, then reloaded
    // four steps ahead, so no register holding a load in flight is copied
    // (a copy would wait for it); the running product alternates between T
    // and T2 for the same reason.
    Aff T, T2, U;
    aff_identity(T);
    float3 w0, w1, w2, w3;
    if (lo < hi) {
        w0 = step_in(lo);
        w1 = step_in(lo + 1);
        w2 = step_in(lo + 2);
        w3 = step_in(lo + 3);
    }
    int s = lo;
    for (; s + 4 <= hi; s += 4) {
        step_u(w0, U);
        w0 = step_in(s + 4);
        aff_compose(U, T, T2);
        step_u(w1, U);
        w1 = step_in(s + 5);
        aff_compose(U, T2, T);
        step_u(w2, U);
        w2 = step_in(s + 6);
        aff_compose(U, T, T2);
        step_u(w3, U);
        w3 = step_in(s + 7);
        aff_compose(U, T2, T);
    }
    for (int k = 0; s < hi; ++s, ++k) {  // the last one to three steps
        step_u(k == 0 ? w0 : (k == 1 ? w1 : w2), U);
        aff_compose(U, T, T2);
        T = T2;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) lds[wave][lane][i] = T.a[i];
    lds[wave][lane][9] = T.b[0];
    lds[wave][lane][10] = T.b[1];
    lds[wave][lane][11] = T.b[2];
    __syncthreads();
    for (int d = 1; d < 64; d <<= 1) {
        Aff L, R, r;
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
            aff_compose(L, R, r);
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
    if (act && lane < 12) j.out[12 * g + lane] = lds[wave][0][lane];
}

hipError_t launch_compose(const RfJobDev *jobs, int n_jobs, int64_t max_groups, double dt,
                          hipStream_t st) {
    if (n_jobs <= 0 || max_groups <= 0) return hipSuccess;
    dim3 grid((unsigned)((max_groups + kComposeGroupsPerWG - 1) / kComposeGroupsPerWG), n_jobs);
    hipLaunchKernelGGL(k_compose, grid, dim3(256), 0, st, jobs, dt);
    return hipGetLastError();
}

// ---------------------------------------------------------------- k_fold
__global__ __launch_bounds__(256) void k_fold(const FoldJob *__restrict__ jobs) {
    const FoldJob j = jobs[blockIdx.y];
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < j.n_groups; g += (int64_t)gridDim.x * 256) {
        Aff T;
#pragma unroll
        for (int i = 0; i < 9; ++i) T.a[i] = j.t64[12 * g + i];
#pragma unroll
        for (int i = 0; i < 3; ++i) T.b[i] = j.t64[12 * g + 9 + i];
        Aff r = T;
        if (j.has_pre) {
            // P: Mxy <- E2 exp(-i phi) Mxy, Mz <- E1 Mz + (1 - E1) M0 (Eq. 4, 5)
            const float4 p = j.gtab[g];  // (coord, T1, T2, df)
            const double cyc = j.cyc * (double)p.x + (double)p.w * j.tau;
            double sn, cs;
            sincos(kTwoPi * (cyc - rint(cyc)), &sn, &cs);
            const double e2 = exp(-j.tau / (double)p.z), e1 = exp(-j.tau / (double)p.y);
            Aff P;
            P.a[0] = e2 * cs;
            P.a[1] = e2 * sn;
            P.a[2] = 0.0;
            P.a[3] = -e2 * sn;
            P.a[4] = e2 * cs;
            P.a[5] = 0.0;
            P.a[6] = 0.0;
            P.a[7] = 0.0;
            P.a[8] = e1;
            P.b[0] = 0.0;
            P.b[1] = 0.0;
            P.b[2] = 1.0 - e1;
            aff_compose(T, P, r);
        }
#pragma unroll
        for (int row = 0; row < 3; ++row)
            j.out[3 * g + row] = make_float4((float)r.a[3 * row], (float)r.a[3 * row + 1], (float)r.a[3 * row + 2],
                                             (float)r.b[row]);
    }
}

hipError_t launch_fold(const FoldJob *jobs, int n_jobs, int64_t max_groups, hipStream_t st) {
    if (n_jobs <= 0 || max_groups <= 0) return hipSuccess;
    int64_t gx = (max_groups + 255) / 256;
    if (gx > 64) gx = 64;
    hipLaunchKernelGGL(k_fold, dim3((unsigned)gx, n_jobs), dim3(256), 0, st, jobs);
    return hipGetLastError();
}

// ---------------------------------------------------------------- k_tables
__global__ __launch_bounds__(256) void k_tables(const TabJob *__restrict__ jobs,
                                                const float4 *__restrict__ gtab_x,
                                                const float4 *__restrict__ gtab_z) {
    const TabJob j = jobs[blockIdx.y];
    for (int g = blockIdx.x * 256 + threadIdx.x; g < j.n; g += gridDim.x * 256) {
        if (j.kind == 0 || j.kind == 2) {
            const float4 p = gtab_x[g];  // (x, T1, T2, df)
            const bool tissue = j.kind == 0;
            const double cyc = j.cyc * (double)p.x + (tissue ? (double)p.w * j.tau : 0.0);
            double sn, cs;
            sincos(kTwoPi * (cyc - rint(cyc)), &sn, &cs);
            const double e2 = tissue ? exp(-j.tau / (double)p.z) : 1.0;
            const double e1 = tissue ? exp(-j.tau / (double)p.y) : 1.0;
            ((float4 *)j.out)[g] = make_float4((float)(e2 * cs), (float)(-e2 * sn), (float)e1, 0.f);
        } else {
            const float4 p = gtab_z[g];
            const double cyc = j.cyc * (double)p.x;
            double sn, cs;
            sincos(kTwoPi * (cyc - rint(cyc)), &sn, &cs);
            ((float2 *)j.out)[g] = make_float2((float)cs, (float)-sn);
        }
    }
}

hipError_t launch_tables(const TabJob *jobs, int n_jobs, int max_n, const float4 *gtab_x,
                         const float4 *gtab_z, hipStream_t st) {
    if (n_jobs <= 0 || max_n <= 0) return hipSuccess;
    int gx = (max_n + 255) / 256;
    if (gx > 64) gx = 64;
    hipLaunchKernelGGL(k_tables, dim3(gx, n_jobs), dim3(256), 0, st, jobs, gtab_x, gtab_z);
    return hipGetLastError();
}

// ---------------------------------------------------------------- k_sweep
// Waves per SIMD the register budgets are sized for: the specialized sweep
// fits its op loop without spills at 5 (96 VGPRs, with the y phases in LDS);
// the general one at 3.
#ifndef SWEEP_NI_FAST
#define SWEEP_NI_FAST 8  // isochromats per thread in the fast sweep
#endif

// The workgroups of a dispatch go to the 8 XCDs round robin (workgroup i to
// XCD i % 8), and each XCD has its own L2.  The sweeps read, at every
// operation, one table row per group of the wavefront (x-group factors,
// transitions); with consecutive slots on different XCDs every XCD fetches
// rows from the whole table, about 1.1 GB per FSE launch.  A sweep grid is
// therefore padded to a multiple of 8 kXcdChunk and the logical blocks are
// dealt to the XCDs in chunks of kXcdChunk consecutive ones: the 16 blocks
// (about 22 x-groups) of a chunk share their rows in one L2, while the
// chunks of one XCD still come from the whole layout, so that regions of
// costlier waves (many small groups) spread over all XCDs.  Logical blocks
// past the end exit at once.
constexpr int kXcds = 8;
constexpr int kXcdChunk = 16;

__device__ __forceinline__ int64_t xcd_block() {
    const int64_t j = blockIdx.x / kXcds, x = blockIdx.x % kXcds;  // j-th workgroup of XCD x
    return ((j / kXcdChunk) * kXcds + x) * kXcdChunk + j % kXcdChunk;
}

static inline unsigned xcd_grid(int64_t blocks) {
    constexpr int64_t q = (int64_t)kXcds * kXcdChunk;
    return (unsigned)(q * ((blocks + q - 1) / q));
}
#ifndef SWEEP_WAVES_FAST
#define SWEEP_WAVES_FAST 5
#endif
#define SWEEP_WAVES_GENERAL 3
#ifndef SWEEP_WAVES_EMIT
#define SWEEP_WAVES_EMIT 6
#endif
constexpr int kSweepMaxCoils = 8;  // receive coils one sweep launch weights (gbs_set_coils' limit)

__device__ __forceinline__ void cmul(float &ar, float &ai, float br, float bi) {
    const float r = ar * br - ai * bi;
    ai = ar * bi + ai * br;
    ar = r;
}

__device__ __forceinline__ void ld4(const float4 *p, int64_t i, float v[4]) {
    const float4 t = p[i];
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
    v[3] = t.w;
}
__device__ __forceinline__ void ld4i(const int4 *p, int64_t i, int v[4]) {
    const int4 t = p[i];
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
    v[3] = t.w;
}

// Table gathers and group-sum atomics through the global address space (the
// pointers come out of op descriptors and would otherwise be flat accesses).
typedef const __attribute__((address_space(1))) float *global_f32_ptr;
__device__ __forceinline__ float4 gather_row(const float4 *tab, int g) {
    global_f32_ptr p = (global_f32_ptr)(tab + g);
    return make_float4(p[0], p[1], p[2], p[3]);
}
__device__ __forceinline__ float2 gather_row(const float2 *tab, int g) {
    global_f32_ptr p = (global_f32_ptr)(tab + g);
    return make_float2(p[0], p[1]);
}
__device__ __forceinline__ void group_add(double *p, double v) {
    __builtin_amdgcn_global_atomic_fadd_f64((__attribute__((address_space(1))) double *)p, v);
}

// Wave-uniform read of a table that no kernel writes while it runs: through
// the constant address space, so a uniform index becomes one scalar load.
typedef const __attribute__((address_space(4))) float *const_f32_ptr;
__device__ __forceinline__ float4 uniform_row(const float4 *tab, int g) {
    const_f32_ptr p = (const_f32_ptr)(tab + g);
    return make_float4(p[0], p[1], p[2], p[3]);
}

typedef const __attribute__((address_space(4))) uint64_t *const_u64_ptr;
static_assert(sizeof(SweepOp) % 8 == 0, "SweepOp is read as 64-bit words");

// The op descriptor is the same for every lane: read it through the constant
// address space so that it arrives in scalar registers.
__device__ __forceinline__ SweepOp load_op(const SweepOp *ops, int o) {
    uint64_t w[sizeof(SweepOp) / 8];
    const_u64_ptr p = (const_u64_ptr)(ops + o);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(SweepOp) / 8); ++i) w[i] = p[i];
    SweepOp r;
    __builtin_memcpy(&r, w, sizeof(SweepOp));
    return r;
}

// x-group row: one scalar load when the wavefront sits inside one x-group.
__device__ __forceinline__ float4 x_row(const float4 *tab, bool gx_uni, int gx0, int gx) {
    return gx_uni ? uniform_row(tab, gx0) : gather_row(tab, gx);
}

// Group sums of (vr, vi) keyed by the thread's group id: one DPP-reduced
// atomic pair when the wavefront has one key, two masked DPP reductions when
// it has two (about a third of the wavefronts straddle one run boundary),
// else a segmented scan over the lanes (keys are sorted runs) and one atomic
// pair per run end.
__device__ __forceinline__ void emit_thread(int key, bool uni, float vr, float vi, bool act,
                                            double2 *__restrict__ gsum) {
    if (uni) {
        vr = wave_sum_lane63(vr);
        vi = wave_sum_lane63(vi);
        if (__lane_id() == 63) {
            group_add(&gsum[key].x, (double)vr);
            group_add(&gsum[key].y, (double)vi);
        }
        return;
    }
    const int k = act ? key : -1;
    // Two runs in the wavefront (or one run and the grid's inactive tail):
    // two masked DPP reductions instead of the segmented scan.
    const int k0 = __builtin_amdgcn_readfirstlane(k), k1 = __builtin_amdgcn_readlane(k, 63);
    if (__all(k == k0 || k == k1)) {
        const bool in0 = k == k0;
        const float ar = wave_sum_lane63(in0 ? vr : 0.f), ai = wave_sum_lane63(in0 ? vi : 0.f);
        const float br = wave_sum_lane63(in0 ? 0.f : vr), bi = wave_sum_lane63(in0 ? 0.f : vi);
        if (__lane_id() == 63) {
            if (k0 >= 0) {
                group_add(&gsum[k0].x, (double)ar);
                group_add(&gsum[k0].y, (double)ai);
            }
            if (k1 >= 0 && k1 != k0) {
                group_add(&gsum[k1].x, (double)br);
                group_add(&gsum[k1].y, (double)bi);
            }
        }
        return;
    }
    const int lane = __lane_id();
    const int kp = __shfl_up(k, 1);
    int head = (lane == 0) || (kp != k);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const float orr = __shfl_up(vr, d);
        const float oi = __shfl_up(vi, d);
        const int oh = __shfl_up(head, d);
        if (lane >= d) {
            if (!head) {
                vr += orr;
                vi += oi;
            }
            head |= oh;
        }
    }
    const int kn = __shfl_down(k, 1);
    if (((lane == 63) || (kn != k)) && k >= 0) {
        group_add(&gsum[k].x, (double)vr);
        group_add(&gsum[k].y, (double)vi);
    }
}

// emit_thread for a kPartials emission: the wavefront's key sums go to its
// float4 entry `part` (first key, other key) instead of memory-side atomics.
__device__ __forceinline__ void emit_thread_part(int key, bool uni, float vr, float vi, bool act, float4 *part,
                                                 double2 *__restrict__ gsum) {
    if (uni) {
        vr = wave_sum_lane63(vr);
        vi = wave_sum_lane63(vi);
        if (__lane_id() == 63) *part = make_float4(vr, vi, 0.f, 0.f);
        return;
    }
    const int k = act ? key : -1;
    const int k0 = __builtin_amdgcn_readfirstlane(k), k1 = __builtin_amdgcn_readlane(k, 63);
    if (__all(k == k0 || k == k1)) {
        const bool in0 = k == k0;
        const float ar = wave_sum_lane63(in0 ? vr : 0.f), ai = wave_sum_lane63(in0 ? vi : 0.f);
        const float br = wave_sum_lane63(in0 ? 0.f : vr), bi = wave_sum_lane63(in0 ? 0.f : vi);
        if (__lane_id() == 63) *part = make_float4(ar, ai, br, bi);
        return;
    }
    if (__lane_id() == 63) *part = make_float4(0.f, 0.f, 0.f, 0.f);
    emit_thread(key, false, vr, vi, act, gsum);
}


// v = v * a + b, the result in v's own register.  The compiler's accumulating
// FMA form would land it in b's register instead, and the state then needs a
// copy back on every pass of the op loop.
__device__ __forceinline__ void fma_inplace(float &v, float a, float b) {
    asm("v_fma_f32 %0, %0, %1, %2" : "+v"(v) : "v"(a), "v"(b));
}

// v = v * a - b in v's own register.
__device__ __forceinline__ void fms_inplace(float &v, float a, float b) {
    asm("v_fma_f32 %0, %0, %1, -%2" : "+v"(v) : "v"(a), "v"(b));
}

// (ar + i ai) <- (ar + i ai)(br + i bi) with the results in ar's and ai's own
// registers, so that a value the loop carries needs no copy.
__device__ __forceinline__ void cmul_inplace(float &ar, float &ai, float br, float bi) {
    const float t = ai * bi, u = ar * bi;
    fma_inplace(ai, br, u);
    fms_inplace(ar, br, t);
}

// M <- T (M, m0) for one isochromat.  Each output's partial sum leaves out
// the diagonal term, so that the last step updates the component in place
// and no copies of the state are needed.
__device__ __forceinline__ void rf_apply(const float4 &r0, const float4 &r1, const float4 &r2, float m0, float &mx,
                                         float &my, float &mz) {
    const float px = fmaf(r0.y, my, fmaf(r0.z, mz, r0.w * m0));
    const float py = fmaf(r1.x, mx, fmaf(r1.z, mz, r1.w * m0));
    const float pz = fmaf(r2.x, mx, fmaf(r2.y, my, r2.w * m0));
    fma_inplace(mx, r0.x, px);
    fma_inplace(my, r1.y, py);
    fma_inplace(mz, r2.z, pz);
}

// rf_apply on the state divided by M0 (see sweep_body): the affine part b
// adds as it is.
__device__ __forceinline__ void rf_apply_ratio(const float4 &r0, const float4 &r1, const float4 &r2, float &mx,
                                               float &my, float &mz) {
    const float px = fmaf(r0.y, my, fmaf(r0.z, mz, r0.w));
    const float py = fmaf(r1.x, mx, fmaf(r1.z, mz, r1.w));
    const float pz = fmaf(r2.x, mx, fmaf(r2.y, my, r2.w));
    fma_inplace(mx, r0.x, px);
    fma_inplace(my, r1.y, py);
    fma_inplace(mz, r2.z, pz);
}

// Row of T applied after the transverse factor f = fr + i fi: the row acting
// on (f (mx + i my)) equals the folded row acting on (mx + i my).
__device__ __forceinline__ void fold_row(float4 &r, float fr, float fi) {
    const float t = r.y * fi, u = r.x * fi;
    fma_inplace(r.x, fr, t);
    fms_inplace(r.y, fr, u);
}

// Real and imaginary parts of sum_c (mx_c + i my_c)(wr_c + i wi_c) as two
// FMA chains per part.
template <int NI>
__device__ __forceinline__ void dot_phase(const float *mx, const float *my, const float *wr, const float *wi,
                                          float &pr, float &pi) {
    float a0 = mx[0] * wr[0], a1 = mx[1] * wr[1];
    float b0 = mx[0] * wi[0], b1 = mx[1] * wi[1];
    a0 = fmaf(-my[0], wi[0], a0);
    a1 = fmaf(-my[1], wi[1], a1);
    b0 = fmaf(my[0], wr[0], b0);
    b1 = fmaf(my[1], wr[1], b1);
#pragma unroll
    for (int c = 2; c < NI; c += 2) {
        a0 = fmaf(mx[c], wr[c], a0);
        a1 = fmaf(mx[c + 1], wr[c + 1], a1);
        b0 = fmaf(mx[c], wi[c], b0);
        b1 = fmaf(mx[c + 1], wi[c + 1], b1);
        a0 = fmaf(-my[c], wi[c], a0);
        a1 = fmaf(-my[c + 1], wi[c + 1], a1);
        b0 = fmaf(my[c], wr[c], b0);
        b1 = fmaf(my[c + 1], wr[c + 1], b1);
    }
    pr = a0 + a1;
    pi = b0 + b1;
}

// FP64 copy of a coordinate for a phase evaluation.  The empty asm keeps the
// compiler from hoisting the conversion out of the op loop, which would hold
// two registers per isochromat for the whole sweep.
__device__ __forceinline__ double coord64(float v) {
    asm volatile("" : "+v"(v));
    return (double)v;
}

// Pairwise sum of N values (N a power of two).
template <int N>
__device__ __forceinline__ float tree_sum(const float *v) {
    float t[N];
#pragma unroll
    for (int c = 0; c < N; ++c) t[c] = v[c];
#pragma unroll
    for (int w = N / 2; w >= 1; w /= 2)
#pragma unroll
        for (int c = 0; c < w; ++c) t[c] += t[c + w];
    return t[0];
}

// Per-isochromat keys (the y axis is not part of the layout's runs).
template <int NI>
__device__ __forceinline__ void emit_items(const int *key, const float *vr, const float *vi, bool act,
                                           double2 *__restrict__ gsum) {
    if (!act) return;
#pragma unroll
    for (int c = 0; c < NI; ++c) {
        group_add(&gsum[key[c]].x, (double)vr[c]);
        group_add(&gsum[key[c]].y, (double)vi[c]);
    }
}

// Each thread owns NI consecutive isochromats of the layout (NI = 4 or 8;
// runs of equal (x-group, z-group) are padded to multiples of 8, so they
// share their x- and z-groups).  GENERAL = false drops what only y-group
// transitions/emissions and direct z phases (no z groups) need, which frees
// registers for occupancy.
template <bool GENERAL, int NI, bool COILS = false, bool PAIRS = false>
__device__ __forceinline__ void sweep_body(const SweepArgs &a) {
    constexpr int NQ = NI / 4;  // float4 words per array and thread
    constexpr int MC = COILS ? kSweepMaxCoils : 1;
    const int64_t blk = xcd_block();
    if (blk * 256 >= a.n4 / NQ) return;  // padding of the XCD grid
    const int64_t it = blk * 256 + threadIdx.x;
    const bool act = it < a.n4 / NQ;
    const int64_t i4 = it * NQ;
    const int need = GENERAL ? a.need : (a.need & ~(kNeedGy | kNeedZ));
    // kPartials: x-emissions write the wavefront's key sums (its 64 threads
    // hold slots 64 NI wave_id ..) instead of memory-side atomics
    constexpr bool PART = !GENERAL && !COILS && NI == SWEEP_NI_FAST;
    const int64_t wave_id = blk * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // RATIO (the fast sweeps that apply transitions): the registers hold
    // M / M0 instead of M.  A combined transition (A, b) then maps M / M0 to
    // A (M / M0) + b, which saves the product b M0 of every row (three per
    // isochromat and transition); M0 is applied where M itself is needed: in
    // the emissions (folded into the y phase factor, which the recurrence
    // carries along) and when the state is written.  An isochromat with
    // M0 = 0 holds 0 (its magnetization is 0 and stays 0; a launch whose
    // initial state is not is routed to the general sweep by the host).
    constexpr bool RATIO = !GENERAL;
    float mx[NI], my[NI], mz[NI], m0[NI], yv[NI], zv[NI];
    int gy[NI];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
        mx[c] = my[c] = mz[c] = m0[c] = yv[c] = zv[c] = 0.f;
        gy[c] = 0;
    }
    int gx = 0, gz = 0, run = 0;
    if (act) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (!a.fresh) {
                ld4(a.mx, i4 + q, mx + 4 * q);
                ld4(a.my, i4 + q, my + 4 * q);
            }
            if (RATIO || (need & kNeedMz)) {
                ld4(a.m0, i4 + q, m0 + 4 * q);
                if (need & kNeedMz) {
                    if (a.fresh) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) mz[4 * q + c] = RATIO ? 1.f : m0[4 * q + c];
                    } else {
                        ld4(a.mz, i4 + q, mz + 4 * q);
                    }
                }
            }
            if (need & kNeedGy) ld4i(a.gid_y, i4 + q, gy + 4 * q);
            if (need & kNeedY) ld4(a.yv, i4 + q, yv + 4 * q);
            if (need & kNeedZ) ld4(a.zv, i4 + q, zv + 4 * q);
        }
        if (RATIO && !a.fresh) {
#pragma unroll
            for (int c = 0; c < NI; ++c) {
                const float inv = m0[c] != 0.f ? 1.f / m0[c] : 0.f;
                mx[c] *= inv;
                my[c] *= inv;
                if (need & kNeedMz) mz[c] *= inv;
            }
        }
        if (need & kNeedGx) gx = a.gid_x[i4].x;
        if (need & kNeedGz) gz = a.gid_z[i4].x;
        if ((GENERAL || PAIRS) && (need & kNeedRun)) run = a.run_of4[i4];  // the thread's slots share a run
    }
    // receive-coil sensitivities of the thread's isochromats, held for the whole launch
    float csr[MC][NI], csi[MC][NI];
#pragma unroll
    for (int p = 0; p < MC; ++p) {
#pragma unroll
        for (int c = 0; c < NI; ++c) csr[p][c] = csi[p][c] = 0.f;
        if (COILS && act && p < a.n_coils) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                ld4(a.coil + 2 * p * a.coil_plane, i4 + q, csr[p] + 4 * q);
                ld4(a.coil + (2 * p + 1) * a.coil_plane, i4 + q, csi[p] + 4 * q);
            }
        }
    }
    // x-groups are contiguous runs in this order: is the wavefront inside one?
    const int gx0 = __builtin_amdgcn_readfirstlane(gx);
    const bool gx_uni = __all(!act || gx == gx0) != 0;
    // y phase of the last emission per isochromat: it changes only at
    // emissions, so it waits in LDS (slot [c][thread]) rather than in registers
    // that would be copied around the op loop.  (rr, ri): its per-step factor.
    __shared__ float2 wsh[NI][256];
    float rr[NI], ri[NI];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
        wsh[c][threadIdx.x] = make_float2(1.f, 0.f);
        rr[c] = 1.f;
        ri[c] = 0.f;
    }

    for (int o = 0; o < a.n_ops; ++o) {
        const SweepOp op = load_op(a.ops, o);
        // a factor common to the thread's isochromats followed by a transition
        // is folded into the thread's rows of T
        bool fold = false;
        float fr = 1.f, fi = 0.f;
        if (op.flags & kOpPre) {
            float e1 = 1.f;
            if (op.pre_xtab) {
                const float4 v = x_row(op.pre_xtab, gx_uni, gx0, gx);
                fr = v.x;
                fi = v.y;
                e1 = v.z;
            }
            if (op.pre_ztab) {
                const float2 v = gather_row(op.pre_ztab, gz);
                cmul(fr, fi, v.x, v.y);
            }
            if (op.pre_cy != 0.0 || (GENERAL && op.pre_cz != 0.0)) {  // per-isochromat phases
                const bool held = (op.flags & (kPreYSet | kPreYHold)) != 0;
                if (op.flags & kPreYSet) {
#pragma unroll
                    for (int c = 0; c < NI; ++c) {
                        float s, co;
                        sincos_rev(op.pre_cy * coord64(yv[c]), &s, &co);
                        rr[c] = co;
                        ri[c] = -s;
                    }
                }
#pragma unroll
                for (int c = 0; c < NI; ++c) {
                    float ar = fr, ai = fi;
                    if (held) {
                        cmul(ar, ai, rr[c], ri[c]);
                    } else if (op.pre_cy != 0.0) {
                        float s, co;
                        sincos_rev(op.pre_cy * coord64(yv[c]), &s, &co);
                        cmul(ar, ai, co, -s);
                    }
                    if (GENERAL && op.pre_cz != 0.0) {
                        float s, co;
                        sincos_rev(op.pre_cz * coord64(zv[c]), &s, &co);
                        cmul(ar, ai, co, -s);
                    }
                    const float nx = mx[c] * ar - my[c] * ai;
                    const float ny = mx[c] * ai + my[c] * ar;
                    mx[c] = nx;
                    my[c] = ny;
                }
            } else if (!(GENERAL && (op.flags & kOpRf) && op.rf_axis == 1)) {
                fold = true;  // into the transition's rows, or into identity rows without one
            } else {  // one factor for all the thread's isochromats
#pragma unroll
                for (int c = 0; c < NI; ++c) {
                    const float nx = mx[c] * fr - my[c] * fi;
                    const float ny = mx[c] * fi + my[c] * fr;
                    mx[c] = nx;
                    my[c] = ny;
                }
            }
            if (op.flags & kPreMz) {
#pragma unroll
                for (int c = 0; c < NI; ++c) mz[c] = RATIO ? fmaf(e1, mz[c] - 1.f, 1.f) : fmaf(e1, mz[c] - m0[c], m0[c]);
            }
        }
        if ((op.flags & kOpRf) || fold) {
            const float4 *__restrict__ tt = op.ttab;
            if (GENERAL && (op.flags & kOpRf) && op.rf_axis == 1) {  // y groups: rows per isochromat
#pragma unroll
                for (int c = 0; c < NI; ++c) {
                    const float4 r0 = gather_row(tt, 3 * gy[c]), r1 = gather_row(tt, 3 * gy[c] + 1),
                                 r2 = gather_row(tt, 3 * gy[c] + 2);
                    const float nx = fmaf(r0.x, mx[c], fmaf(r0.y, my[c], fmaf(r0.z, mz[c], r0.w * m0[c])));
                    const float ny = fmaf(r1.x, mx[c], fmaf(r1.y, my[c], fmaf(r1.z, mz[c], r1.w * m0[c])));
                    const float nz = fmaf(r2.x, mx[c], fmaf(r2.y, my[c], fmaf(r2.z, mz[c], r2.w * m0[c])));
                    mx[c] = nx;
                    my[c] = ny;
                    mz[c] = nz;
                }
            } else {
                float4 r0, r1, r2;
                if (!(op.flags & kOpRf)) {
                    r0 = make_float4(1.f, 0.f, 0.f, 0.f);
                    r1 = make_float4(0.f, 1.f, 0.f, 0.f);
                    r2 = make_float4(0.f, 0.f, 1.f, 0.f);
                } else if (op.rf_axis == 0 && gx_uni) {
                    r0 = uniform_row(tt, 3 * gx0);
                    r1 = uniform_row(tt, 3 * gx0 + 1);
                    r2 = uniform_row(tt, 3 * gx0 + 2);
                } else {
                    const int g = op.rf_axis == 0 ? gx : ((GENERAL || PAIRS) && op.rf_axis == 3 ? run : gz);
                    r0 = gather_row(tt, 3 * g);
                    r1 = gather_row(tt, 3 * g + 1);
                    r2 = gather_row(tt, 3 * g + 2);
                }
                if (fold) {
                    fold_row(r0, fr, fi);
                    fold_row(r1, fr, fi);
                    fold_row(r2, fr, fi);
                }
#pragma unroll
                for (int c = 0; c < NI; ++c) {
                    if (RATIO)
                        rf_apply_ratio(r0, r1, r2, mx[c], my[c], mz[c]);
                    else
                        rf_apply(r0, r1, r2, m0[c], mx[c], my[c], mz[c]);
                }
            }
        }
        if (op.flags & kOpEmit) {
            const float4 xv = x_row(op.emit_xtab, gx_uni, gx0, gx);
            float er = xv.x, ei = xv.y;
            // the z row is gathered first and used last, so that the gather's
            // latency overlaps the y phase and the sum (fast sweep)
            float2 zf = make_float2(1.f, 0.f);
            if (op.emit_ztab) zf = gather_row(op.emit_ztab, gz);
            if (GENERAL && op.emit_ztab) cmul(er, ei, zf.x, zf.y);
            // y phase of this emission: evaluated, or stepped from the last one
            const bool yph = (op.flags & (kYDirect | kYStep)) != 0;
            auto y_phase = [&](float *wr, float *wi) {
                if (op.flags & kYDirect) {
#pragma unroll
                    for (int c = 0; c < NI; ++c) {
                        float s, co;
                        sincos_rev(op.emit_cy * coord64(yv[c]), &s, &co);
                        wr[c] = RATIO ? co * m0[c] : co;  // RATIO: the factor carries M0
                        wi[c] = RATIO ? -s * m0[c] : -s;
                        wsh[c][threadIdx.x] = make_float2(wr[c], wi[c]);
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < NI; ++c) {
                        const float2 w = wsh[c][threadIdx.x];
                        wr[c] = w.x;
                        wi[c] = w.y;
                        cmul(wr[c], wi[c], rr[c], ri[c]);
                        wsh[c][threadIdx.x] = make_float2(wr[c], wi[c]);
                    }
                }
            };
            if (GENERAL && (COILS || op.emit_cz != 0.0 || op.emit_axis == 1)) {
                float wr[NI], wi[NI], vr[NI], vi[NI];
                if (yph) y_phase(wr, wi);
#pragma unroll
                for (int c = 0; c < NI; ++c) {
                    float ar = er, ai = ei;
                    if (yph) cmul(ar, ai, wr[c], wi[c]);
                    if (op.emit_cz != 0.0) {
                        float s, co;
                        sincos_rev(op.emit_cz * coord64(zv[c]), &s, &co);
                        cmul(ar, ai, co, -s);
                    }
                    vr[c] = mx[c] * ar - my[c] * ai;
                    vi[c] = mx[c] * ai + my[c] * ar;
                }
                if (COILS) {  // every coil: members weighted by S(k, p), then its own group sums
#pragma unroll
                    for (int p = 0; p < MC; ++p) {
                        if (p >= a.n_coils) break;
                        float ur[NI], ui[NI];
#pragma unroll
                        for (int c = 0; c < NI; ++c) {
                            ur[c] = vr[c] * csr[p][c] - vi[c] * csi[p][c];
                            ui[c] = vr[c] * csi[p][c] + vi[c] * csr[p][c];
                        }
                        double2 *gs = op.gsum + (int64_t)p * op.gsum_stride;
                        if (op.emit_axis == 1) {
                            emit_items<NI>(gy, ur, ui, act, gs);
                        } else {
                            const float sr = tree_sum<NI>(ur), si = tree_sum<NI>(ui);
                            if (op.emit_axis == 0)
                                emit_thread(gx_uni ? gx0 : gx, gx_uni, sr, si, act, gs);
                            else
                                emit_thread(gz, false, sr, si, act, gs);
                        }
                    }
                } else if (op.emit_axis == 1) {
                    emit_items<NI>(gy, vr, vi, act, op.gsum);
                } else {
                    const float sr = tree_sum<NI>(vr), si = tree_sum<NI>(vi);
                    if (op.emit_axis == 0 && PART && (need & kPartials))
                        emit_thread_part(gx_uni ? gx0 : gx, gx_uni, sr, si, act, op.part + wave_id, op.gsum);
                    else if (op.emit_axis == 0)
                        emit_thread(gx_uni ? gx0 : gx, gx_uni, sr, si, act, op.gsum);
                    else
                        emit_thread(gz, false, sr, si, act, op.gsum);
                }
            } else {
                // the factor of the x and z groups is common to the thread's
                // isochromats: sum (M_c w_c) first, multiply once
                float pr, pi;
                if (yph) {
                    float wr[NI], wi[NI];
                    y_phase(wr, wi);
                    dot_phase<NI>(mx, my, wr, wi, pr, pi);
                } else if (RATIO) {
                    float tx[NI], ty[NI];
#pragma unroll
                    for (int c = 0; c < NI; ++c) {
                        tx[c] = mx[c] * m0[c];
                        ty[c] = my[c] * m0[c];
                    }
                    pr = tree_sum<NI>(tx);
                    pi = tree_sum<NI>(ty);
                } else {
                    pr = tree_sum<NI>(mx);
                    pi = tree_sum<NI>(my);
                }
                if (!GENERAL && op.emit_ztab) cmul(er, ei, zf.x, zf.y);
                const float sr = er * pr - ei * pi, si = er * pi + ei * pr;
                if (op.emit_axis == 0 && PART && (need & kPartials))
                    emit_thread_part(gx_uni ? gx0 : gx, gx_uni, sr, si, act, op.part + wave_id, op.gsum);
                else if (op.emit_axis == 0)
                    emit_thread(gx_uni ? gx0 : gx, gx_uni, sr, si, act, op.gsum);
                else
                    emit_thread(gz, false, sr, si, act, op.gsum);
            }
            if (op.flags & kYSetR) {  // step factor of the chain this emission starts
#pragma unroll
                for (int c = 0; c < NI; ++c) {
                    float s, co;
                    sincos_rev(op.emit_dcy * coord64(yv[c]), &s, &co);
                    rr[c] = co;
                    ri[c] = -s;
                }
            }
        }
    }
    if (RATIO && act && a.write_m) {  // back to M
#pragma unroll
        for (int c = 0; c < NI; ++c) {
            mx[c] *= m0[c];
            my[c] *= m0[c];
            mz[c] *= m0[c];
        }
    }
    if (act && a.write_m && a.m_final) {
#pragma unroll
        for (int c = 0; c < NI; ++c) a.m_final[4 * i4 + c] = make_float4(mx[c], my[c], mz[c], 0.f);
    } else if (act && a.write_m) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            a.mx[i4 + q] = make_float4(mx[4 * q], mx[4 * q + 1], mx[4 * q + 2], mx[4 * q + 3]);
            a.my[i4 + q] = make_float4(my[4 * q], my[4 * q + 1], my[4 * q + 2], my[4 * q + 3]);
            if (need & kNeedMz) a.mz[i4 + q] = make_float4(mz[4 * q], mz[4 * q + 1], mz[4 * q + 2], mz[4 * q + 3]);
        }
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SWEEP_WAVES_FAST))) void k_sweep(SweepArgs a) {
    sweep_body<false, SWEEP_NI_FAST>(a);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SWEEP_WAVES_GENERAL))) void k_sweep_general(
    SweepArgs a) {
    sweep_body<true, 4>(a);
}

// The fast sweep for runs with two-axis (x, z) transitions: rows per run of
// the layout (a thread's 8 slots lie in one run).  The run index is one
// register more than the fast sweep holds at 5 waves per SIMD, so 4.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_pairs(
    SweepArgs a) {
    sweep_body<false, SWEEP_NI_FAST, false, true>(a);
}

// The sweep for segments whose ops only emit (an EPI readout train).  The
// state does not change between the emissions, so each thread holds its M_c
// for the whole launch and carries z_c = M_c w_c, w_c being the y phase of
// the current emission (Eq. 8-9 with the accumulated blip moments).  A chain
// of evenly stepped emissions (its first op carries the count of the
// stepped ones that follow) starts with a direct evaluation of w_c (M_c waits
// in LDS for these chain starts, slot [c][thread]) and then
// multiplies z_c by the step factor r_c in place, so each further emission
// costs one complex product and the sum of the z_c per isochromat.  Each
// emission scales the thread's sum by its x- and z-group factors.  Ops
// before the emissions that change the state (kEmitHead: the excitation and
// the pre map of the first readout) are applied once, first, and a closed
// form map that ends the segment (kEmitTail) once, after the emissions.
template <int NI>
__device__ __forceinline__ void emit_sweep_body(const SweepArgs &a) {
    constexpr int NQ = NI / 4;
    const int64_t blk = xcd_block();
    if (blk * 256 >= a.n4 / NQ) return;  // padding of the XCD grid
    const int64_t it = blk * 256 + threadIdx.x;
    const bool act = it < a.n4 / NQ;
    const int64_t i4 = it * NQ;
    const int need = a.need;
    __shared__ float2 msh[NI][256];
    __shared__ float msz[NI][256];  // Mz after the head ops (kEmitHead)
    float yv[NI];
    int gx = 0, gz = 0, gx0 = 0;
    bool gx_uni = true;
    const int64_t wave_id = blk * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // slots 512 wave_id ..
    // the x- and z-group factor rows of an emission
    auto emit_rows = [&](const SweepOp &op, float4 &xv, float2 &zf) {
        xv = x_row(op.emit_xtab, gx_uni, gx0, gx);
        zf = op.emit_ztab ? gather_row(op.emit_ztab, gz) : make_float2(1.f, 0.f);
    };
    // one emission from the thread's sum (pr, pi) of M_c w_c: x- and z-group
    // factors (rows already loaded), then the group sums
    auto emit_sum_rows = [&](const SweepOp &op, const float4 &xv, const float2 &zf, float pr, float pi) {
        float er = xv.x, ei = xv.y;
        if (op.emit_ztab) cmul(er, ei, zf.x, zf.y);
        const float sr = er * pr - ei * pi, si = er * pi + ei * pr;
        if (op.emit_axis == 0 && (need & kPartials))
            emit_thread_part(gx_uni ? gx0 : gx, gx_uni, sr, si, act, op.part + wave_id, op.gsum);
        else if (op.emit_axis == 0)
            emit_thread(gx_uni ? gx0 : gx, gx_uni, sr, si, act, op.gsum);
        else
            emit_thread(gz, false, sr, si, act, op.gsum);
    };
    auto emit_sum = [&](const SweepOp &op, float pr, float pi) {
        float4 xv;
        float2 zf;
        emit_rows(op, xv, zf);
        emit_sum_rows(op, xv, zf, pr, pi);
    };
    {
        float mx[NI], my[NI];
#pragma unroll
        for (int c = 0; c < NI; ++c) mx[c] = my[c] = yv[c] = 0.f;
        if (act) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (!a.fresh) {
                    ld4(a.mx, i4 + q, mx + 4 * q);
                    ld4(a.my, i4 + q, my + 4 * q);
                }
                if (need & kNeedY) ld4(a.yv, i4 + q, yv + 4 * q);
            }
            if (need & kNeedGx) gx = a.gid_x[i4].x;
            if (need & kNeedGz) gz = a.gid_z[i4].x;
        }
        gx0 = __builtin_amdgcn_readfirstlane(gx);
        gx_uni = __all(!act || gx == gx0) != 0;
        if (need & kEmitHead) {  // general ops before the emissions, with the whole state in registers
            float mz[NI], m0[NI];
#pragma unroll
            for (int c = 0; c < NI; ++c) mz[c] = m0[c] = 0.f;
            if (act && (need & kNeedMz)) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    ld4(a.m0, i4 + q, m0 + 4 * q);
                    ld4(a.fresh ? a.m0 : a.mz, i4 + q, mz + 4 * q);
                }
            }
            for (int o = 0; o < a.n_head; ++o) {
                const SweepOp op = load_op(a.ops, o);
                if (op.flags & kOpPre) {  // Eq. 4, 5 by group factors and the direct y phase
                    float fr = 1.f, fi = 0.f, e1 = 1.f;
                    if (op.pre_xtab) {
                        const float4 v = x_row(op.pre_xtab, gx_uni, gx0, gx);
                        fr = v.x;
                        fi = v.y;
                        e1 = v.z;
                    }
                    if (op.pre_ztab) {
                        const float2 v = gather_row(op.pre_ztab, gz);
                        cmul(fr, fi, v.x, v.y);
                    }
#pragma unroll
                    for (int c = 0; c < NI; ++c) {
                        float ar = fr, ai = fi;
                        if (op.pre_cy != 0.0) {
                            float sn, co;
                            sincos_rev(op.pre_cy * coord64(yv[c]), &sn, &co);
                            cmul(ar, ai, co, -sn);
                        }
                        cmul(mx[c], my[c], ar, ai);
                        if (op.flags & kPreMz) mz[c] = fmaf(e1, mz[c] - m0[c], m0[c]);
                    }
                }
                if (op.flags & kOpRf) {  // the group's combined transition (Eq. 7)
                    float4 r0, r1, r2;
                    if (op.rf_axis == 0 && gx_uni) {
                        r0 = uniform_row(op.ttab, 3 * gx0);
                        r1 = uniform_row(op.ttab, 3 * gx0 + 1);
                        r2 = uniform_row(op.ttab, 3 * gx0 + 2);
                    } else {
                        const int g = op.rf_axis == 0 ? gx : gz;
                        r0 = gather_row(op.ttab, 3 * g);
                        r1 = gather_row(op.ttab, 3 * g + 1);
                        r2 = gather_row(op.ttab, 3 * g + 2);
                    }
#pragma unroll
                    for (int c = 0; c < NI; ++c) rf_apply(r0, r1, r2, m0[c], mx[c], my[c], mz[c]);
                }
                if (op.flags & kOpEmit) {  // (no chain crosses into the emissions that follow)
                    float wr[NI], wi[NI];
#pragma unroll
                    for (int c = 0; c < NI; ++c) {
                        float sn = 0.f, co = 1.f;
                        if (op.flags & kYDirect) sincos_rev(op.emit_cy * coord64(yv[c]), &sn, &co);
                        wr[c] = mx[c] * co + my[c] * sn;
                        wi[c] = my[c] * co - mx[c] * sn;
                    }
                    emit_sum(op, tree_sum<NI>(wr), tree_sum<NI>(wi));
                }
            }
#pragma unroll
            for (int c = 0; c < NI; ++c) msz[c][threadIdx.x] = mz[c];
        }
#pragma unroll
        for (int c = 0; c < NI; ++c) msh[c][threadIdx.x] = make_float2(mx[c], my[c]);
    }
    float zr[NI], zi[NI], rr[NI], ri[NI];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
        zr[c] = zi[c] = ri[c] = 0.f;
        rr[c] = 1.f;
    }
    auto emit = [&](const SweepOp &op) { emit_sum(op, tree_sum<NI>(zr), tree_sum<NI>(zi)); };
    const int n_emit = a.n_ops - ((need & kEmitTail) ? 1 : 0);
    for (int o = (need & kEmitHead) ? a.n_head : 0; o < n_emit;) {
        const SweepOp op = load_op(a.ops, o++);
        if (op.flags & kYDirect) {
#pragma unroll
            for (int c = 0; c < NI; ++c) {
                float sn, co;
                sincos_rev(op.emit_cy * coord64(yv[c]), &sn, &co);
                const float2 m = msh[c][threadIdx.x];
                zr[c] = m.x * co + m.y * sn;  // M (co - i sn)
                zi[c] = m.y * co - m.x * sn;
            }
        } else if (op.flags & kYStep) {
#pragma unroll
            for (int c = 0; c < NI; ++c) cmul_inplace(zr[c], zi[c], rr[c], ri[c]);
        } else {
#pragma unroll
            for (int c = 0; c < NI; ++c) {
                const float2 m = msh[c][threadIdx.x];
                zr[c] = m.x;
                zi[c] = m.y;
            }
        }
        emit(op);
        if (op.flags & kYSetR) {  // step factor of the chain this emission starts
#pragma unroll
            for (int c = 0; c < NI; ++c) {
                float sn, co;
                sincos_rev(op.emit_dcy * coord64(yv[c]), &sn, &co);
                rr[c] = co;
                ri[c] = -sn;
            }
        }
        // the evenly stepped emissions of the chain, software-pipelined: the
        // next op's descriptor is loaded before this emission's arithmetic and
        // its factor rows right after this emission, so neither latency sits
        // in front of the work that needs it (indices are clamped into the
        // segment; the loads past the chain's end are never used)
        const int steps = min((op.flags >> kChainShift) & kChainMask, n_emit - o);
        if (steps > 0) {
            SweepOp sop = load_op(a.ops, o);
            float4 xv;
            float2 zf;
            emit_rows(sop, xv, zf);
            for (int j = 0; j < steps; ++j) {
                const SweepOp nxt = load_op(a.ops, min(o + 1, n_emit - 1));
#pragma unroll
                for (int c = 0; c < NI; ++c) cmul_inplace(zr[c], zi[c], rr[c], ri[c]);
                emit_sum_rows(sop, xv, zf, tree_sum<NI>(zr), tree_sum<NI>(zi));
                ++o;
                emit_rows(nxt, xv, zf);
                sop = nxt;
            }
        }
    }
    if (!act || !a.write_m) return;
    float mx[NI], my[NI], mz[NI], m0[NI];
#pragma unroll
    for (int c = 0; c < NI; ++c) {
        const float2 m = msh[c][threadIdx.x];
        mx[c] = m.x;
        my[c] = m.y;
        mz[c] = m0[c] = 0.f;
    }
    if (need & kEmitHead) {  // Mz as the head ops left it
#pragma unroll
        for (int c = 0; c < NI; ++c) mz[c] = msz[c][threadIdx.x];
    } else if (need & kNeedMz) {  // Mz is unchanged: (0, 0, M0) or as read
#pragma unroll
        for (int q = 0; q < NQ; ++q) ld4(a.fresh ? a.m0 : a.mz, i4 + q, mz + 4 * q);
    }
    if (need & kEmitTail) {  // the closed-form map that ends the segment (Eq. 4, 5)
        const SweepOp op = load_op(a.ops, a.n_ops - 1);
        float fr = 1.f, fi = 0.f, e1 = 1.f;
        if (op.pre_xtab) {
            const float4 v = x_row(op.pre_xtab, gx_uni, gx0, gx);
            fr = v.x;
            fi = v.y;
            e1 = v.z;
        }
        if (op.pre_ztab) {
            const float2 v = gather_row(op.pre_ztab, gz);
            cmul(fr, fi, v.x, v.y);
        }
#pragma unroll
        for (int c = 0; c < NI; ++c) {
            float ar = fr, ai = fi;
            if (op.pre_cy != 0.0) {
                float sn, co;
                sincos_rev(op.pre_cy * coord64(yv[c]), &sn, &co);
                cmul(ar, ai, co, -sn);
            }
            const float nx = mx[c] * ar - my[c] * ai;
            const float ny = mx[c] * ai + my[c] * ar;
            mx[c] = nx;
            my[c] = ny;
        }
        if (op.flags & kPreMz) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) ld4(a.m0, i4 + q, m0 + 4 * q);
#pragma unroll
            for (int c = 0; c < NI; ++c) mz[c] = fmaf(e1, mz[c] - m0[c], m0[c]);
        }
    }
    if (a.m_final) {
#pragma unroll
        for (int c = 0; c < NI; ++c) a.m_final[4 * i4 + c] = make_float4(mx[c], my[c], mz[c], 0.f);
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            a.mx[i4 + q] = make_float4(mx[4 * q], mx[4 * q + 1], mx[4 * q + 2], mx[4 * q + 3]);
            a.my[i4 + q] = make_float4(my[4 * q], my[4 * q + 1], my[4 * q + 2], my[4 * q + 3]);
            if (need & kNeedMz) a.mz[i4 + q] = make_float4(mz[4 * q], mz[4 * q + 1], mz[4 * q + 2], mz[4 * q + 3]);
        }
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SWEEP_WAVES_EMIT))) void k_sweep_emit(
    SweepArgs a) {
    emit_sweep_body<SWEEP_NI_FAST>(a);
}

// The general sweep with receive coils: the thread's sensitivities (up to
// kSweepMaxCoils coils) stay in registers for the whole launch.
__global__ __launch_bounds__(256) void k_sweep_coils(SweepArgs a) { sweep_body<true, 4, true>(a); }

hipError_t launch_sweep(const SweepArgs &a, hipStream_t st) {
    if (a.n4 <= 0 || a.n_ops <= 0) return hipSuccess;
    if (a.n4 % (SWEEP_NI_FAST / 4)) return hipErrorInvalidValue;  // the layout pads runs to multiples of 8
    if (a.coil) {
        if (a.n_coils < 1 || a.n_coils > kSweepMaxCoils) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_sweep_coils, dim3(xcd_grid((a.n4 + 255) / 256)), dim3(256), 0, st, a);
    } else if (a.need & (kNeedGy | kNeedZ | kForceGeneral)) {
        hipLaunchKernelGGL(k_sweep_general, dim3(xcd_grid((a.n4 + 255) / 256)), dim3(256), 0, st, a);
    } else {
        const int64_t n = a.n4 / (SWEEP_NI_FAST / 4);
        if (a.need & kEmitOnly)
            hipLaunchKernelGGL(k_sweep_emit, dim3(xcd_grid((n + 255) / 256)), dim3(256), 0, st, a);
        else if (a.need & kNeedRun)
            hipLaunchKernelGGL(k_sweep_pairs, dim3(xcd_grid((n + 255) / 256)), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL(k_sweep, dim3(xcd_grid((n + 255) / 256)), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- k_adc_eval
constexpr int kAdcChunk = 1024;  // groups per workgroup

__global__ void k_adc_eval(const AdcJobDev *__restrict__ jobs, double *__restrict__ sig_base) {
    const AdcJobDev j = jobs[blockIdx.y];
    double *sig = sig_base + 2 * j.sig_offset;
    const int g0 = blockIdx.x * kAdcChunk;
    if (g0 >= j.n_groups) return;
    const int g1 = min(g0 + kAdcChunk, j.n_groups);
    for (int n = threadIdx.x; n < j.n_samples; n += blockDim.x) {
        const double2 sm = j.samp[n];  // (tau_n, gamma_bar * m_n)
        const float tauf = (float)sm.x;
        double ar = 0.0, ai = 0.0;
        for (int g = g0; g < g1; ++g) {
            const float4 p = j.gtab[g];  // (coord, T1, T2, df)
            const double2 S = j.gsum[g];
            const double cyc = sm.y * (double)p.x + (double)p.w * sm.x;
            float s, c;
            sincos_rev(cyc, &s, &c);
            const float e = __expf(-tauf * __builtin_amdgcn_rcpf(p.z));
            const double tr = (double)(e * c), ti = (double)(-e * s);
            ar = fma(tr, S.x, fma(-ti, S.y, ar));
            ai = fma(tr, S.y, fma(ti, S.x, ai));
        }
        atomicAdd(&sig[2 * n], ar);
        atomicAdd(&sig[2 * n + 1], ai);
    }
}

hipError_t launch_adc_eval(const AdcJobDev *jobs, int n_jobs, int max_groups, int max_samples,
                           double *sig, hipStream_t st) {
    if (n_jobs <= 0 || max_groups <= 0 || max_samples <= 0) return hipSuccess;
    int bs = ((max_samples + 63) / 64) * 64;
    if (bs > 256) bs = 256;
    dim3 grid((max_groups + kAdcChunk - 1) / kAdcChunk, n_jobs);
    hipLaunchKernelGGL(k_adc_eval, grid, dim3(bs), 0, st, jobs, sig);
    return hipGetLastError();
}

// ---------------------------------------------------------------- layout helpers
__global__ void k_fill_f64(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_fill_f64(double *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)g), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

__global__ void k_init_state(int64_t K, int64_t Kpad, const int32_t *__restrict__ perm,
                             const float *__restrict__ ix, const float *__restrict__ iy,
                             const float *__restrict__ iz, const float *__restrict__ m0i,
                             float *__restrict__ mx, float *__restrict__ my, float *__restrict__ mz) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Kpad; i += (int64_t)gridDim.x * blockDim.x) {
        float x = 0.f, y = 0.f, z = 0.f;
        const int32_t k = i < K ? perm[i] : -1;  // -1: padding of the group-sorted layout
        if (k >= 0) {
            if (ix) {
                x = ix[k];
                y = iy[k];
                z = iz[k];
            } else {
                z = m0i[i];
            }
        }
        mx[i] = x;
        my[i] = y;
        mz[i] = z;
    }
}

hipError_t launch_init_state(int64_t K, int64_t Kpad, const int32_t *perm, const float *mi_x,
                             const float *mi_y, const float *mi_z, const float *m0i, float *mx,
                             float *my, float *mz, hipStream_t st) {
    int64_t g = (Kpad + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_init_state, dim3((unsigned)g), dim3(256), 0, st, K, Kpad, perm, mi_x, mi_y,
                       mi_z, m0i, mx, my, mz);
    return hipGetLastError();
}

// Final state in the caller's order: coalesced writes, reads through the
// inverse permutation (neighbouring caller indices usually sit in nearby
// rows of the group-sorted layout, so the reads hit L2).
__global__ void k_gather_state(int64_t K, const int32_t *__restrict__ inv, const float *__restrict__ mx,
                               const float *__restrict__ my, const float *__restrict__ mz, float *ox, float *oy,
                               float *oz) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = inv[k];
        ox[k] = mx[i];
        oy[k] = my[i];
        oz[k] = mz[i];
    }
}

// Workgroups go to the 8 XCDs in turn, and each XCD has its own L2.  Caller
// indices one grid row apart (same x and z) sit in neighbouring slots of one
// run of the layout, i.e. in one cache line of the 16-byte rows, so each XCD
// takes a contiguous range of caller indices: the line's four rows are then
// read through one L2 instead of being fetched once per XCD.

__global__ __launch_bounds__(256) void k_gather_state4(int64_t K, int64_t per_xcd, const int32_t *__restrict__ inv,
                                                      const float4 *__restrict__ m4, float *ox, float *oy,
                                                      float *oz) {
    const int64_t b = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;  // logical block
    const int64_t k = b * 256 + threadIdx.x;
    if (k < K) {
        const float4 v = m4[inv[k]];
        ox[k] = v.x;
        oy[k] = v.y;
        oz[k] = v.z;
    }
}

// Four caller indices per thread: one 16-byte index load, four independent
// row gathers in flight, 16-byte stores.  Needs K % 4 == 0 and 16-byte
// aligned planes.
__global__ __launch_bounds__(256) void k_gather_state4x4(int64_t K4, int64_t per_xcd, const int4 *__restrict__ inv4,
                                                        const float4 *__restrict__ m4, float4 *ox, float4 *oy,
                                                        float4 *oz) {
    const int64_t b = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;  // logical block
    const int64_t k = b * 256 + threadIdx.x;
    if (k < K4) {
        const int4 r = inv4[k];
        const float4 a = m4[r.x], c = m4[r.y], d = m4[r.z], e = m4[r.w];
        ox[k] = make_float4(a.x, c.x, d.x, e.x);
        oy[k] = make_float4(a.y, c.y, d.y, e.y);
        oz[k] = make_float4(a.z, c.z, d.z, e.z);
    }
}

hipError_t launch_gather_state4(int64_t K, const int32_t *inv, const float4 *m4, float *ox, float *oy, float *oz,
                                hipStream_t st) {
    const bool by4 = K % 4 == 0 && ((uintptr_t)ox | (uintptr_t)inv) % 16 == 0;  // oy, oz = ox + K, + 2K
    const int64_t n = by4 ? K / 4 : K;   // threads
    const int64_t g = (n + 255) / 256;   // logical blocks
    const int64_t per = (g + kXcds - 1) / kXcds;
    if (kXcds * per > 0x7fffffff) return hipErrorInvalidValue;
    if (g == 0) return hipSuccess;
    if (by4)
        hipLaunchKernelGGL(k_gather_state4x4, dim3((unsigned)(kXcds * per)), dim3(256), 0, st, n, per,
                           (const int4 *)inv, m4, (float4 *)ox, (float4 *)oy, (float4 *)oz);
    else
        hipLaunchKernelGGL(k_gather_state4, dim3((unsigned)(kXcds * per)), dim3(256), 0, st, K, per, inv, m4, ox, oy,
                           oz);
    return hipGetLastError();
}

// gsum[g] += sum of the partial entries of the wavefronts that span x-group g
// (kPartials), one thread per group and kPartJobsPerThread emissions, FP64
// sums.  A wavefront's entry holds its first key's sum in (x, y) and its other
// key's in (z, w).  Every wavefront after the first of the group starts
// inside the group, so g is its first key; the first one has g first only if
// g starts at the wavefront's first slot.  The group's bounds are read once;
// the emissions' first entries are all loaded before any is added (job
// indices clamped into the launch; a clamped duplicate is never written back).
constexpr int kPartJobsPerThread = 4;
typedef const __attribute__((address_space(1))) float4 *part_gptr;
typedef __attribute__((address_space(1))) double2 *gsum_gptr;

__global__ __launch_bounds__(256) void k_part_reduce(const PartJob *__restrict__ jobs, int n_jobs, int64_t n_groups,
                                                    const int32_t *__restrict__ xstart) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= n_groups) return;
    const int64_t s0 = xstart[g];
    const int64_t w0 = s0 / kPartSlots, w1 = (xstart[g + 1] - 1) / kPartSlots;
    const bool head = s0 % kPartSlots == 0;
    const int j0 = blockIdx.y * kPartJobsPerThread;
    part_gptr part[kPartJobsPerThread];
    float4 v0[kPartJobsPerThread];
#pragma unroll
    for (int q = 0; q < kPartJobsPerThread; ++q) {
        part[q] = (part_gptr)jobs[min(j0 + q, n_jobs - 1)].part;
        v0[q] = part[q][w0];
    }
#pragma unroll
    for (int q = 0; q < kPartJobsPerThread; ++q) {
        double sr = head ? v0[q].x : v0[q].z, si = head ? v0[q].y : v0[q].w;
        for (int64_t w = w0 + 1; w <= w1; ++w) {
            const float4 v = part[q][w];
            sr += v.x;
            si += v.y;
        }
        if (j0 + q < n_jobs) {
            gsum_gptr gs = (gsum_gptr)jobs[j0 + q].gsum + g;
            double2 t = *gs;
            t.x += sr;
            t.y += si;
            *gs = t;
        }
    }
}

hipError_t launch_part_reduce(const PartJob *jobs, int n_jobs, int64_t n_groups, const int32_t *xstart,
                              hipStream_t st) {
    if (n_jobs <= 0 || n_groups <= 0) return hipSuccess;
    const int gy = (n_jobs + kPartJobsPerThread - 1) / kPartJobsPerThread;
    if (gy > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_part_reduce, dim3((unsigned)((n_groups + 255) / 256), (unsigned)gy), dim3(256), 0, st, jobs,
                       n_jobs, n_groups, xstart);
    return hipGetLastError();
}

__global__ void k_group_starts(int64_t n, const int32_t *__restrict__ gid_x, int64_t n_groups,
                               int32_t *__restrict__ xstart) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        if (i == n)
            xstart[n_groups] = (int32_t)n;
        else if (i == 0 || gid_x[i - 1] != gid_x[i])
            xstart[gid_x[i]] = (int32_t)i;
    }
}

hipError_t launch_group_starts(int64_t n, const int32_t *gid_x, int64_t n_groups, int32_t *xstart, hipStream_t st) {
    int64_t g = (n + 256) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_group_starts, dim3((unsigned)g), dim3(256), 0, st, n, gid_x, n_groups, xstart);
    return hipGetLastError();
}

__global__ void k_check_zero_m0(int64_t K, const float *__restrict__ m0, const float *__restrict__ mx,
                                const float *__restrict__ my, const float *__restrict__ mz, int *flag) {
    bool bad = false;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x)
        bad = bad || (m0[k] == 0.f && (mx[k] != 0.f || my[k] != 0.f || mz[k] != 0.f));
    if (__any(bad) && __lane_id() == 0) *flag = 1;
}

hipError_t launch_check_zero_m0(int64_t K, const float *m0, const float *mx, const float *my, const float *mz,
                                int *flag, hipStream_t st) {
    int64_t g = (K + 255) / 256;
    if (g > 4096) g = 4096;
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_zero_m0, dim3((unsigned)g), dim3(256), 0, st, K, m0, mx, my, mz, flag);
    return hipGetLastError();
}

hipError_t launch_gather_state(int64_t K, const int32_t *inv, const float *mx, const float *my, const float *mz,
                               float *ox, float *oy, float *oz, hipStream_t st) {
    int64_t g = (K + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_gather_state, dim3((unsigned)g), dim3(256), 0, st, K, inv, mx, my, mz, ox, oy, oz);
    return hipGetLastError();
}

}  // namespace gbs
