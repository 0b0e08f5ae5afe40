// Two-axis (x, z) groups on gfx950: the runs of the group-sorted layout and
// one combined transition per run for Gx+Gz with-RF subsequences.
//
// k_compose_pair: one thread per run composes its 3x4 homogeneous transition
// in FP64 (the same product as the per-isochromat composition of the cached
// method, with the run's x, z, T1, T2, dB0); the step's waveform values are
// wave-uniform scalar loads.
#include "consts.hpp"
#include "pairs.hpp"
#include "rotation.hpp"

namespace gbs {

__global__ void k_run_flags(int64_t n4, const int32_t *__restrict__ gid_x, const int32_t *__restrict__ gid_z,
                            uint8_t *__restrict__ flag) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += (int64_t)gridDim.x * blockDim.x)
        flag[q] = q == 0 || gid_x[4 * q] != gid_x[4 * q - 4] || gid_z[4 * q] != gid_z[4 * q - 4];
}

__global__ void k_run_table(int64_t n_runs, const int32_t *__restrict__ first, const float *__restrict__ xi,
                            const float *__restrict__ zi, const float *__restrict__ t1i,
                            const float *__restrict__ t2i, const float *__restrict__ dfi, float4 *__restrict__ rtab,
                            float *__restrict__ rz) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_runs;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = 4 * (int64_t)first[r];  // a run starts with a real isochromat
        rtab[r] = make_float4(xi[k], t1i[k], t2i[k], dfi[k]);
        rz[r] = zi[k];
    }
}

__global__ __launch_bounds__(256) void k_compose_pair(int64_t n_runs, const float4 *__restrict__ rtab,
                                                      const float *__restrict__ rz, const StepW *__restrict__ wave,
                                                      int32_t n_steps, double dt, double *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n_runs) return;
    const float4 g = rtab[r];
    const double X = g.x, Z = rz[r], t1 = g.y, t2 = g.z;
    const double boff = (double)g.w / kGammaBar;
    const double e1 = exp(-dt / t1), e2 = exp(-dt / t2), e1m = -expm1(-dt / t1);
    const double gdt = kTwoPi * kGammaBar * dt, k2 = gdt * gdt;
    double T[3][4] = {{1.0, 0.0, 0.0, 0.0}, {0.0, 1.0, 0.0, 0.0}, {0.0, 0.0, 1.0, 0.0}}, U[3][4];
    // V = (D R)_j V0 for raster step j, then the T1 recovery toward M0
    auto step = [&](const double (&V0)[3][4], double (&V)[3][4], int j) {
        const StepW w = wave[j];
        const double bx = w.b1r, by = w.b1i;
        const double bz = fma((double)w.gx, X, fma((double)w.gz, Z, boff));
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
    // two steps per iteration, T -> U -> T: the loop carries no register
    // copies of the twelve entries
    int j = 0;
    for (; j + 1 < n_steps; j += 2) {
        step(T, U, j);
        step(U, T, j + 1);
    }
    if (j < n_steps) {
        step(T, U, j);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) T[i][c] = U[i][c];
    }
    double *o = out + 12 * r;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int c = 0; c < 3; ++c) o[3 * i + c] = T[i][c];
        o[9 + i] = T[i][3];
    }
}

static dim3 grid_of(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return dim3((unsigned)g);
}

hipError_t launch_run_flags(int64_t n4, const int32_t *gid_x, const int32_t *gid_z, uint8_t *flag, hipStream_t st) {
    if (n4 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_run_flags, grid_of(n4), dim3(256), 0, st, n4, gid_x, gid_z, flag);
    return hipGetLastError();
}

hipError_t launch_run_table(int64_t n_runs, const int32_t *first, const float *xi, const float *zi,
                            const float *t1i, const float *t2i, const float *dfi, float4 *rtab, float *rz,
                            hipStream_t st) {
    if (n_runs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_run_table, grid_of(n_runs), dim3(256), 0, st, n_runs, first, xi, zi, t1i, t2i, dfi, rtab, rz);
    return hipGetLastError();
}

hipError_t launch_compose_pair(int64_t n_runs, const float4 *rtab, const float *rz, const StepW *wave,
                               int32_t n_steps, double dt, double *out, hipStream_t st) {
    if (n_runs <= 0) return hipSuccess;
    const int64_t blocks = (n_runs + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_compose_pair, dim3((unsigned)blocks), dim3(256), 0, st, n_runs, rtab, rz, wave, n_steps,
                       dt, out);
    return hipGetLastError();
}

}  // namespace gbs
