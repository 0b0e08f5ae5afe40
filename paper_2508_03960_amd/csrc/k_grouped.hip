// Grouped-isochromat kernels for gfx950 (Sec. 2.3, 2.4).
//
//  k_compose   combined transition T = U_{N-1} ... U_0 (Eq. 7) once per group,
//              FP64.  One wavefront per group: each lane composes a contiguous
//              chunk of steps, then the 64 partial products are combined in a
//              log2 tree through LDS (later chunk on the left).
//  k_tables    per-group factors of the closed-form B1 = 0 maps (Eq. 4, 5):
//              x-groups carry decay, off-resonance and x phase; z-groups the
//              z phase.
//  k_sweep     one coalesced sweep over the group-sorted isochromats that
//              applies a run of grouped operations with the state in
//              registers: pre maps, group transitions, and the group sums of
//              each with-ADC subsequence (Eq. 9) reduced across the wavefront
//              (one group per wavefront in the common case), then FP64 atomics.
//  k_adc_eval  every ADC sample from the group sums (Eq. 8 with Eq. 10), FP64
//              phase reduced to a quarter turn, FP64 accumulation.
#include "device_math.hpp"
#include "kernels.hpp"

namespace gbs {

// ---------------------------------------------------------------- k_compose
constexpr int kComposeGroupsPerWG = 4;

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
    const int n = j.n_steps;
    const int lo = (int)(((int64_t)n * lane) >> 6), hi = (int)(((int64_t)n * (lane + 1)) >> 6);
    Aff T;
    aff_identity(T);
    for (int s = lo; s < hi; ++s) {
        const StepW w = j.wave[s];
        const double gv = j.axis == 0 ? w.gx : (j.axis == 1 ? w.gy : w.gz);
        const double bx = w.b1r, by = w.b1i, bz = gv * coord + boff;
        const double nb = sqrt(bx * bx + by * by + bz * bz);
        Aff U;  // U = D R (Eq. A1, Eq. A2)
        if (nb == 0.0) {
            aff_identity(U);
        } else {
            const double ux = bx / nb, uy = by / nb, uz = bz / nb;
            const double th = -kTwoPi * kGammaBar * nb * dt;
            double sn, cs;
            sincos(th, &sn, &cs);
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
            U.b[0] = U.b[1] = U.b[2] = 0.0;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            U.a[c] *= e2;
            U.a[3 + c] *= e2;
            U.a[6 + c] *= e1;
        }
        U.b[2] = 1.0 - e1;
        Aff Tn;
        aff_compose(U, T, Tn);
        T = Tn;
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
    if (act && lane < 3) {
        const double *row = &lds[wave][0][0];
        j.out[3 * g + lane] = make_float4((float)row[3 * lane], (float)row[3 * lane + 1],
                                          (float)row[3 * lane + 2], (float)row[9 + lane]);
    }
}

hipError_t launch_compose(const RfJobDev *jobs, int n_jobs, int64_t max_groups, double dt,
                          hipStream_t st) {
    if (n_jobs <= 0 || max_groups <= 0) return hipSuccess;
    dim3 grid((unsigned)((max_groups + kComposeGroupsPerWG - 1) / kComposeGroupsPerWG), n_jobs);
    hipLaunchKernelGGL(k_compose, grid, dim3(256), 0, st, jobs, dt);
    return hipGetLastError();
}

// ---------------------------------------------------------------- k_tables
__global__ __launch_bounds__(256) void k_tables(const TabJob *__restrict__ jobs,
                                                const float4 *__restrict__ gtab_x,
                                                const float4 *__restrict__ gtab_z) {
    const TabJob j = jobs[blockIdx.y];
    for (int g = blockIdx.x * 256 + threadIdx.x; g < j.n; g += gridDim.x * 256) {
        if (j.kind == 0) {
            const float4 p = gtab_x[g];  // (x, T1, T2, df)
            const double cyc = j.cyc * (double)p.x + (double)p.w * j.tau;
            const double ph = kTwoPi * (cyc - rint(cyc));
            double sn, cs;
            sincos(ph, &sn, &cs);
            const double e2 = exp(-j.tau / (double)p.z), e1 = exp(-j.tau / (double)p.y);
            ((float4 *)j.out)[g] = make_float4((float)(e2 * cs), (float)(-e2 * sn), (float)e1, 0.f);
        } else {
            const float4 p = gtab_z[g];
            const double cyc = j.cyc * (double)p.x;
            const double ph = kTwoPi * (cyc - rint(cyc));
            double sn, cs;
            sincos(ph, &sn, &cs);
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

// ---------------------------------------------------------------- k_pass
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

__device__ __forceinline__ bool same4(const int g[4]) { return g[0] == g[1] && g[0] == g[2] && g[0] == g[3]; }

// Wave-uniform read of a table that no kernel writes while it runs: through
// the constant address space, so a uniform index becomes one scalar load.
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

typedef const __attribute__((address_space(4))) float *const_f32_ptr;
__device__ __forceinline__ float4 uniform_row(const float4 *tab, int g) {
    const_f32_ptr p = (const_f32_ptr)(tab + g);
    return make_float4(p[0], p[1], p[2], p[3]);
}
__device__ __forceinline__ float2 uniform_row(const float2 *tab, int g) {
    const_f32_ptr p = (const_f32_ptr)(tab + g);
    return make_float2(p[0], p[1]);
}

// Table rows of the thread's 4 isochromats.  Group ids are sorted runs, so
// the whole wavefront usually shares one x-group (one scalar load) and a
// thread's 4 neighbours usually share their other groups (one gather).
template <class T>
__device__ __forceinline__ void rows4(const T *__restrict__ tab, const int g[4], bool wave_uniform, int g_uni,
                                      T out[4]) {
    if (wave_uniform) {
        const T v = uniform_row(tab, g_uni);
        out[0] = out[1] = out[2] = out[3] = v;
    } else if (same4(g)) {
        const T v = gather_row(tab, g[0]);
        out[0] = out[1] = out[2] = out[3] = v;
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) out[c] = gather_row(tab, g[c]);
    }
}

// Mxy factor a and E1 of a B1 = 0 map for the thread's 4 isochromats.
__device__ __forceinline__ void map_factor4(const MapTabs &m, const int gx[4], bool gx_uni, int gx0,
                                            const int gz[4], const float y[4], const float z[4],
                                            float ar[4], float ai[4], float e1[4]) {
    float4 xf[4];
    rows4(m.xtab, gx, gx_uni, gx0, xf);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        ar[c] = xf[c].x;
        ai[c] = xf[c].y;
        e1[c] = xf[c].z;
    }
    if (m.ztab) {
        float2 zf[4];
        rows4(m.ztab, gz, false, 0, zf);
#pragma unroll
        for (int c = 0; c < 4; ++c) cmul(ar[c], ai[c], zf[c].x, zf[c].y);
    }
    if (m.cy != 0.0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            float s, co;
            sincos_rev(m.cy * (double)y[c], &s, &co);
            cmul(ar[c], ai[c], co, -s);
        }
    }
    if (m.cz != 0.0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            float s, co;
            sincos_rev(m.cz * (double)z[c], &s, &co);
            cmul(ar[c], ai[c], co, -s);
        }
    }
}

// Sum (vr, vi) per run of equal keys: within the thread, then across the
// wavefront with a segmented inclusive scan; segment ends add to gsum.
__device__ __forceinline__ void emit_runs(const int key[4], const float vr[4], const float vi[4],
                                          bool act, double2 *__restrict__ gsum) {
    int k = act ? key[0] : -1;
    double sr = 0.0, si = 0.0;
    if (act) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (key[c] != k) {
                group_add(&gsum[k].x, sr);
                group_add(&gsum[k].y, si);
                sr = si = 0.0;
                k = key[c];
            }
            sr += (double)vr[c];
            si += (double)vi[c];
        }
    }
    const int lane = __lane_id();
    const int kp = __shfl_up(k, 1);
    int head = (lane == 0) || (kp != k);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double orr = __shfl_up(sr, d);
        const double oi = __shfl_up(si, d);
        const int oh = __shfl_up(head, d);
        if (lane >= d) {
            if (!head) {
                sr += orr;
                si += oi;
            }
            head |= oh;
        }
    }
    const int kn = __shfl_down(k, 1);
    const bool tail = (lane == 63) || (kn != k);
    if (tail && k >= 0) {
        group_add(&gsum[k].x, sr);
        group_add(&gsum[k].y, si);
    }
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

__global__ __launch_bounds__(256) void k_sweep(SweepArgs a) {
    const int64_t i4 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool act = i4 < a.n4;
    const int need = a.need;
    float mx[4] = {0, 0, 0, 0}, my[4] = {0, 0, 0, 0}, mz[4] = {0, 0, 0, 0}, m0[4] = {0, 0, 0, 0};
    float yv[4] = {0, 0, 0, 0}, zv[4] = {0, 0, 0, 0};
    int gx[4] = {-1, -1, -1, -1}, gy[4] = {0, 0, 0, 0}, gz[4] = {0, 0, 0, 0};
    if (act) {
        ld4(a.mx, i4, mx);
        ld4(a.my, i4, my);
        if (need & kNeedMz) {
            ld4(a.mz, i4, mz);
            ld4(a.m0, i4, m0);
        }
        if (need & kNeedGx) ld4i(a.gid_x, i4, gx);
        if (need & kNeedGy) ld4i(a.gid_y, i4, gy);
        if (need & kNeedGz) ld4i(a.gid_z, i4, gz);
        if (need & kNeedY) ld4(a.yv, i4, yv);
        if (need & kNeedZ) ld4(a.zv, i4, zv);
    }
    // x-groups are contiguous runs in this order: is the wavefront inside one?
    const int gx0 = __builtin_amdgcn_readfirstlane(gx[0]);
    const bool gx_uni = __all(act && same4(gx) && gx[0] == gx0) != 0;
    const int gxs[4] = {act ? gx[0] : 0, act ? gx[1] : 0, act ? gx[2] : 0, act ? gx[3] : 0};

    for (int o = 0; o < a.n_ops; ++o) {
        const SweepOp op = load_op(a.ops, o);
        if (op.flags & kOpPre) {
            float ar[4], ai[4], e1[4];
            map_factor4(op.pre, gxs, gx_uni, gx0, gz, yv, zv, ar, ai, e1);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float nx = mx[c] * ar[c] - my[c] * ai[c];
                const float ny = mx[c] * ai[c] + my[c] * ar[c];
                mx[c] = nx;
                my[c] = ny;
                mz[c] = fmaf(e1[c], mz[c] - m0[c], m0[c]);
            }
        }
        if (op.flags & kOpRf) {
            const int *grf = op.rf_axis == 0 ? gxs : (op.rf_axis == 1 ? gy : gz);
            const float4 *__restrict__ tt = op.ttab;
            float4 r0[4], r1[4], r2[4];
            if (op.rf_axis == 0 && gx_uni) {
                const float4 u0 = uniform_row(tt, 3 * gx0), u1 = uniform_row(tt, 3 * gx0 + 1),
                             u2 = uniform_row(tt, 3 * gx0 + 2);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    r0[c] = u0;
                    r1[c] = u1;
                    r2[c] = u2;
                }
            } else if (same4(grf)) {
                const int g = grf[0];
                const float4 u0 = gather_row(tt, 3 * g), u1 = gather_row(tt, 3 * g + 1),
                             u2 = gather_row(tt, 3 * g + 2);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    r0[c] = u0;
                    r1[c] = u1;
                    r2[c] = u2;
                }
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    r0[c] = gather_row(tt, 3 * grf[c]);
                    r1[c] = gather_row(tt, 3 * grf[c] + 1);
                    r2[c] = gather_row(tt, 3 * grf[c] + 2);
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float nx = fmaf(r0[c].x, mx[c], fmaf(r0[c].y, my[c], fmaf(r0[c].z, mz[c], r0[c].w * m0[c])));
                const float ny = fmaf(r1[c].x, mx[c], fmaf(r1[c].y, my[c], fmaf(r1[c].z, mz[c], r1[c].w * m0[c])));
                const float nz = fmaf(r2[c].x, mx[c], fmaf(r2[c].y, my[c], fmaf(r2[c].z, mz[c], r2[c].w * m0[c])));
                mx[c] = nx;
                my[c] = ny;
                mz[c] = nz;
            }
        }
        if (op.flags & kOpEmit) {
            float ar[4], ai[4], e1[4], vr[4], vi[4];
            map_factor4(op.emit, gxs, gx_uni, gx0, gz, yv, zv, ar, ai, e1);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                vr[c] = act ? mx[c] * ar[c] - my[c] * ai[c] : 0.f;
                vi[c] = act ? mx[c] * ai[c] + my[c] * ar[c] : 0.f;
            }
            if (op.emit_axis == 0 && gx_uni) {
                // one group for the whole wavefront: DPP sum, one FP64 atomic pair
                float sr = (vr[0] + vr[1]) + (vr[2] + vr[3]);
                float si = (vi[0] + vi[1]) + (vi[2] + vi[3]);
                sr = wave_sum_lane63(sr);
                si = wave_sum_lane63(si);
                if (__lane_id() == 63) {
                    group_add(&op.gsum[gx0].x, (double)sr);
                    group_add(&op.gsum[gx0].y, (double)si);
                }
            } else {
                int key[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) key[c] = op.emit_axis == 0 ? gxs[c] : (op.emit_axis == 1 ? gy[c] : gz[c]);
                emit_runs(key, vr, vi, act, op.gsum);
            }
        }
    }
    if (act && a.write_m) {
        a.mx[i4] = make_float4(mx[0], mx[1], mx[2], mx[3]);
        a.my[i4] = make_float4(my[0], my[1], my[2], my[3]);
        if (need & kNeedMz) a.mz[i4] = make_float4(mz[0], mz[1], mz[2], mz[3]);
    }
}

hipError_t launch_sweep(const SweepArgs &a, hipStream_t st) {
    if (a.n4 <= 0 || a.n_ops <= 0) return hipSuccess;
    const int64_t grid = (a.n4 + 255) / 256;
    hipLaunchKernelGGL(k_sweep, dim3((unsigned)grid), dim3(256), 0, st, a);
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
        if (i < K) {
            if (ix) {
                const int32_t k = perm[i];
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

__global__ void k_scatter_state(int64_t K, const int32_t *__restrict__ perm, const float *__restrict__ mx,
                                const float *__restrict__ my, const float *__restrict__ mz,
                                float *ox, float *oy, float *oz) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = perm[i];
        ox[k] = mx[i];
        oy[k] = my[i];
        oz[k] = mz[i];
    }
}

hipError_t launch_scatter_state(int64_t K, const int32_t *perm, const float *mx, const float *my,
                                const float *mz, float *ox, float *oy, float *oz, hipStream_t st) {
    int64_t g = (K + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_scatter_state, dim3((unsigned)g), dim3(256), 0, st, K, perm, mx, my, mz, ox,
                       oy, oz);
    return hipGetLastError();
}

}  // namespace gbs
