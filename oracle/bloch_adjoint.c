/*
 * FP64 CPU oracle of the gradient of the k-space signal (TEST INFRASTRUCTURE
 * ONLY: used by the test suite and the benchmark's CPU leg, never by the GPU
 * library, and sharing no code with it).
 *
 * Forward model: the plain per-isochromat simulation (Eq. 2 with U = D R of
 * Eq. A1 and Eq. A2 per raster step; Eq. 4 and Eq. 5 for relaxation blocks;
 * Eq. 6 for the signal).  Parameters: the complex B1 samples of the
 * "parameter pulse" (n_rf samples, used by every block listed in
 * param_blocks in place of its own B1), and per-class T1 and T2 (every
 * isochromat carries a class index).
 *
 * Scalar objective: L = sum_n (w_re[n] Re A_n + w_im[n] Im A_n) for a given
 * cotangent w of the signal A.  Reverse mode written out: the state of every
 * boundary is stored in the forward pass; going backward, lambda_p (dL/dM at
 * boundary p) gains the cotangents of the samples taken at p and is carried
 * through each step by the transpose of its 3x3 Jacobian.  The derivative of
 * a step map with respect to a parameter is taken by the complex step
 * (f(x + i h) has imaginary part h f'(x) + O(h^3)), with h = 1e-30, on the
 * same formulas as the forward model evaluated in complex arithmetic.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AJ_GAMMA_BAR 42.577478518e6
#define AJ_TWO_PI 6.283185307179586476925286766559005768
#define AJ_H 1e-30

typedef double complex cplx;

/* One raster step (Eq. A2 then Eq. A1) on a real state, complex parameters. */
static void step_c(const double M[3], double m0, cplx bx, cplx by, cplx bz, cplx t1, cplx t2, double dt,
                   cplx out[3])
{
    cplx R[9];
    cplx nb2 = bx * bx + by * by + bz * bz;
    if (creal(nb2) == 0.0 && cimag(nb2) == 0.0) {
        for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
    } else {
        cplx nb = csqrt(nb2);
        cplx ux = bx / nb, uy = by / nb, uz = bz / nb;
        cplx th = -AJ_TWO_PI * AJ_GAMMA_BAR * nb * dt;
        cplx c = ccos(th), s = csin(th), v = 1.0 - c;
        R[0] = c + ux * ux * v;
        R[1] = -uz * s + ux * uy * v;
        R[2] = uy * s + ux * uz * v;
        R[3] = uz * s + ux * uy * v;
        R[4] = c + uy * uy * v;
        R[5] = -ux * s + uy * uz * v;
        R[6] = -uy * s + ux * uz * v;
        R[7] = ux * s + uy * uz * v;
        R[8] = c + uz * uz * v;
    }
    cplx e1 = cexp(-dt / t1), e2 = cexp(-dt / t2);
    cplx v0 = R[0] * M[0] + R[1] * M[1] + R[2] * M[2];
    cplx v1 = R[3] * M[0] + R[4] * M[1] + R[5] * M[2];
    cplx v2 = R[6] * M[0] + R[7] * M[1] + R[8] * M[2];
    out[0] = e2 * v0;
    out[1] = e2 * v1;
    out[2] = e1 * v2 + (1.0 - e1) * m0;
}

/* Relaxation block (Eq. 4, Eq. 5): phase in FP64 reduced modulo one turn. */
static void relax_c(const double M[3], double m0, double cycles, double tau, cplx t1, cplx t2, cplx out[3])
{
    double ph = AJ_TWO_PI * (cycles - nearbyint(cycles));
    double c = cos(ph), s = sin(ph);
    cplx e1 = cexp(-tau / t1), e2 = cexp(-tau / t2);
    out[0] = e2 * (M[0] * c + M[1] * s);
    out[1] = e2 * (M[1] * c - M[0] * s);
    out[2] = e1 * M[2] + (1.0 - e1) * m0;
}

typedef struct {
    int kind;     /* 0 raster step, 1 relaxation */
    int64_t w;    /* raster: waveform index */
    int32_t par;  /* raster: parameter-pulse sample, or -1 */
    double tau;   /* relaxation */
    double mom[3];
} aj_op;

int oracle_adjoint(int64_t K, const double *x, const double *y, const double *z, const double *df,
                   const double *m0, const int32_t *cls, int32_t n_classes, const double *t1c,
                   const double *t2c, int64_t n_blocks, const int32_t *btype, const int64_t *step_offset,
                   const int64_t *n_steps, const int64_t *n_samples, const int64_t *sample_offset,
                   const double *tau, const double *moment, int64_t total_steps, const double *rf_re,
                   const double *rf_im, const double *gx, const double *gy, const double *gz,
                   int64_t total_samples, const int32_t *adc_idx, double dt, int64_t n_rf,
                   const int32_t *param_blocks, int32_t n_param_blocks, const double *rf_param,
                   const double *w, int nthreads, double *sig_out, double *g_rf, double *g_t1, double *g_t2)
{
    if (K < 0 || n_blocks < 0 || n_classes < 1 || !(dt > 0.0)) return -1;
    /* flatten the blocks into ops and per-boundary sample lists */
    int64_t n_ops = 0;
    for (int64_t b = 0; b < n_blocks; ++b) {
        if (btype[b] != 3 && (n_steps[b] < 0 || n_steps[b] > ((int64_t)1 << 32))) return -1;
        n_ops += (btype[b] == 3) ? 1 : n_steps[b];
    }
    if (n_ops < 0 || n_ops > ((int64_t)1 << 36)) return -1;
    aj_op *ops = (aj_op *)calloc((size_t)(n_ops > 0 ? n_ops : 1), sizeof(aj_op));
    int64_t *sstart = (int64_t *)calloc((size_t)(n_ops + 2), sizeof(int64_t));
    int64_t *sid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total_samples > 0 ? total_samples : 1));
    int64_t *spos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total_samples > 0 ? total_samples : 1));
    if (!ops || !sstart || !sid || !spos) return -2;
    int64_t o = 0;
    for (int64_t b = 0; b < n_blocks; ++b) {
        if (btype[b] == 3) {
            ops[o].kind = 1;
            ops[o].tau = tau[b];
            for (int i = 0; i < 3; ++i) ops[o].mom[i] = moment[3 * b + i];
            ++o;
            continue;
        }
        int par = 0;
        for (int32_t q = 0; q < n_param_blocks; ++q) par |= (param_blocks[q] == b);
        if (par && n_steps[b] != n_rf) return -1;
        for (int64_t n = 0; n < n_samples[b]; ++n) spos[sample_offset[b] + n] = o + adc_idx[sample_offset[b] + n];
        for (int64_t j = 0; j < n_steps[b]; ++j, ++o) {
            ops[o].kind = 0;
            ops[o].w = step_offset[b] + j;
            ops[o].par = par ? (int32_t)j : -1;
        }
    }
    for (int64_t n = 0; n < total_samples; ++n) sstart[spos[n] + 1]++;
    for (int64_t p = 0; p <= n_ops; ++p) sstart[p + 1] += sstart[p];
    {
        int64_t *fill = (int64_t *)calloc((size_t)(n_ops + 1), sizeof(int64_t));
        for (int64_t n = 0; n < total_samples; ++n) sid[sstart[spos[n]] + fill[spos[n]]++] = n;
        free(fill);
    }
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    int nt = 1;
    (void)nthreads;
#endif
    const size_t nsig = 2 * (size_t)total_samples, nrf = 2 * (size_t)n_rf;
    double *p_sig = (double *)calloc((size_t)nt * (nsig + 1), sizeof(double));
    double *p_rf = (double *)calloc((size_t)nt * (nrf + 1), sizeof(double));
    double *p_t = (double *)calloc((size_t)nt * 2 * (size_t)n_classes, sizeof(double));
    int bad = 0;
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *S = (double *)malloc(sizeof(double) * 3 * (size_t)(n_ops + 1));
        double *ms = p_sig + (size_t)tid * (nsig + 1), *mr = p_rf + (size_t)tid * (nrf + 1);
        double *mt = p_t + (size_t)tid * 2 * (size_t)n_classes;
        if (!S) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(static)
        for (int64_t k = 0; k < K; ++k) {
            if (!S) continue;
            const int c = cls[k];
            if (c < 0 || c >= n_classes) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            const double T1 = t1c[c], T2 = t2c[c];
            S[0] = 0.0;
            S[1] = 0.0;
            S[2] = m0[k];
            /* forward: states at every boundary, samples */
            for (int64_t p = 0; p <= n_ops; ++p) {
                for (int64_t q = sstart[p]; q < sstart[p + 1]; ++q) {
                    ms[2 * sid[q]] += S[3 * p];
                    ms[2 * sid[q] + 1] += S[3 * p + 1];
                }
                if (p == n_ops) break;
                const aj_op *op = &ops[p];
                cplx out[3];
                if (op->kind == 1) {
                    double cyc = AJ_GAMMA_BAR * (op->mom[0] * x[k] + op->mom[1] * y[k] + op->mom[2] * z[k]) +
                                 df[k] * op->tau;
                    relax_c(&S[3 * p], m0[k], cyc, op->tau, T1, T2, out);
                } else {
                    double bx = op->par >= 0 ? rf_param[2 * op->par] : rf_re[op->w];
                    double by = op->par >= 0 ? rf_param[2 * op->par + 1] : rf_im[op->w];
                    double bz = gx[op->w] * x[k] + gy[op->w] * y[k] + gz[op->w] * z[k] + df[k] / AJ_GAMMA_BAR;
                    step_c(&S[3 * p], m0[k], bx, by, bz, T1, T2, dt, out);
                }
                for (int i = 0; i < 3; ++i) S[3 * (p + 1) + i] = creal(out[i]);
            }
            /* backward */
            double lam[3] = {0.0, 0.0, 0.0};
            for (int64_t p = n_ops; p >= 0; --p) {
                for (int64_t q = sstart[p]; q < sstart[p + 1]; ++q) {
                    lam[0] += w[2 * sid[q]];
                    lam[1] += w[2 * sid[q] + 1];
                }
                if (p == 0) break;
                const aj_op *op = &ops[p - 1];
                const double *Mi = &S[3 * (p - 1)];
                cplx d[3];
                double J[9];
                if (op->kind == 1) {
                    double cyc = AJ_GAMMA_BAR * (op->mom[0] * x[k] + op->mom[1] * y[k] + op->mom[2] * z[k]) +
                                 df[k] * op->tau;
                    relax_c(Mi, m0[k], cyc, op->tau, T1 + I * AJ_H, T2, d);
                    mt[2 * c] += (lam[0] * cimag(d[0]) + lam[1] * cimag(d[1]) + lam[2] * cimag(d[2])) / AJ_H;
                    relax_c(Mi, m0[k], cyc, op->tau, T1, T2 + I * AJ_H, d);
                    mt[2 * c + 1] += (lam[0] * cimag(d[0]) + lam[1] * cimag(d[1]) + lam[2] * cimag(d[2])) / AJ_H;
                    for (int j = 0; j < 3; ++j) {  /* Jacobian columns: the map is affine in M */
                        double e[3] = {0.0, 0.0, 0.0};
                        e[j] = 1.0;
                        relax_c(e, 0.0, cyc, op->tau, T1, T2, d);
                        for (int i = 0; i < 3; ++i) J[3 * i + j] = creal(d[i]);
                    }
                } else {
                    double bx = op->par >= 0 ? rf_param[2 * op->par] : rf_re[op->w];
                    double by = op->par >= 0 ? rf_param[2 * op->par + 1] : rf_im[op->w];
                    double bz = gx[op->w] * x[k] + gy[op->w] * y[k] + gz[op->w] * z[k] + df[k] / AJ_GAMMA_BAR;
                    step_c(Mi, m0[k], bx, by, bz, T1 + I * AJ_H, T2, dt, d);
                    mt[2 * c] += (lam[0] * cimag(d[0]) + lam[1] * cimag(d[1]) + lam[2] * cimag(d[2])) / AJ_H;
                    step_c(Mi, m0[k], bx, by, bz, T1, T2 + I * AJ_H, dt, d);
                    mt[2 * c + 1] += (lam[0] * cimag(d[0]) + lam[1] * cimag(d[1]) + lam[2] * cimag(d[2])) / AJ_H;
                    if (op->par >= 0) {
                        step_c(Mi, m0[k], bx + I * AJ_H, by, bz, T1, T2, dt, d);
                        mr[2 * op->par] += (lam[0] * cimag(d[0]) + lam[1] * cimag(d[1]) + lam[2] * cimag(d[2])) / AJ_H;
                        step_c(Mi, m0[k], bx, by + I * AJ_H, bz, T1, T2, dt, d);
                        mr[2 * op->par + 1] +=
                            (lam[0] * cimag(d[0]) + lam[1] * cimag(d[1]) + lam[2] * cimag(d[2])) / AJ_H;
                    }
                    for (int j = 0; j < 3; ++j) {
                        double e[3] = {0.0, 0.0, 0.0};
                        e[j] = 1.0;
                        step_c(e, 0.0, bx, by, bz, T1, T2, dt, d);
                        for (int i = 0; i < 3; ++i) J[3 * i + j] = creal(d[i]);
                    }
                }
                double nl[3];
                for (int j = 0; j < 3; ++j) nl[j] = J[j] * lam[0] + J[3 + j] * lam[1] + J[6 + j] * lam[2];
                lam[0] = nl[0];
                lam[1] = nl[1];
                lam[2] = nl[2];
            }
        }
        free(S);
    }
    if (!bad) {
        memset(sig_out, 0, sizeof(double) * nsig);
        memset(g_rf, 0, sizeof(double) * nrf);
        memset(g_t1, 0, sizeof(double) * (size_t)n_classes);
        memset(g_t2, 0, sizeof(double) * (size_t)n_classes);
        for (int t = 0; t < nt; ++t) { /* fixed thread order: deterministic */
            for (size_t i = 0; i < nsig; ++i) sig_out[i] += p_sig[(size_t)t * (nsig + 1) + i];
            for (size_t i = 0; i < nrf; ++i) g_rf[i] += p_rf[(size_t)t * (nrf + 1) + i];
            for (int c = 0; c < n_classes; ++c) {
                g_t1[c] += p_t[(size_t)t * 2 * n_classes + 2 * c];
                g_t2[c] += p_t[(size_t)t * 2 * n_classes + 2 * c + 1];
            }
        }
    }
    free(p_sig);
    free(p_rf);
    free(p_t);
    free(ops);
    free(sstart);
    free(sid);
    free(spos);
    return bad ? -1 : 0;
}
