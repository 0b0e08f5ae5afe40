/*
 * FP64 CPU oracle: plain per-isochromat Bloch simulation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant with the GPU library.
 *
 * What it computes (H. Takeshima, "Fast Magnetic Resonance Simulation Using
 * Combined Update with Grouped Isochromats"):
 *
 *  - every isochromat k starts at M = (0, 0, M0(k)) unless an initial state
 *    is given, and carries the homogeneous 4-vector (Mx, My, Mz, M0) (Eq. 2);
 *  - in RF and ADC blocks it is advanced raster step by raster step with the
 *    4x4 transition U = D * R (Appendix A, asymmetric operator splitting:
 *    rotation first, then relaxation).  B is piecewise constant over a step:
 *    B = (Re B1, Im B1, G . r + dB0) (Sec. 2.1).  R is the Rodrigues rotation
 *    of Eq. (A2) about u = B/|B| by theta = -gamma |B| dt, the identity when
 *    |B| = 0; D is Eq. (A1);
 *  - a relaxation block of duration tau and gradient moment m = int G dt is
 *    applied with the closed forms Eq. (4) and Eq. (5):
 *      Mxy <- Mxy exp(-tau/T2) exp(-i (gamma m . r + 2 pi df tau)),
 *      Mz  <- M0 + (Mz - M0) exp(-tau/T1);
 *  - ADC sample n of a block adds Mx + i My of every isochromat, at the raster
 *    boundary adc_idx[n] of that block, to the k-space sample (Eq. 6 with one
 *    coil of unit sensitivity).
 *
 * Readings of the paper taken here:
 *  - relaxation decays toward M0 (the sign in Eq. (1) is garbled; Eq. (4),
 *    Eq. (5) and Eq. (A1) fix the decaying direction);
 *  - gamma/2pi = 42.577478518 MHz/T; the field inhomogeneity is given in Hz,
 *    so B_z gains df/(gamma/2pi) tesla;
 *  - phases of relaxation blocks are reduced modulo one cycle in FP64.
 *
 * Threads: OpenMP over isochromats with a static schedule; each thread sums
 * its own signal partials, and the partials are added in thread order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_GAMMA_BAR 42.577478518e6 /* Hz/T */
#define OR_TWO_PI 6.283185307179586476925286766559005768

enum { OR_BLOCK_RF = 1, OR_BLOCK_ADC = 2, OR_BLOCK_RELAX = 3 };

enum { OR_OK = 0, OR_E_INVALID = -1, OR_E_NOMEM = -4 };

/* Eq. (A2): rotation by theta = -gamma |B| dt about u = B/|B|. */
static void rotation_matrix(double bx, double by, double bz, double dt, double R[4][4])
{
    memset(R, 0, 16 * sizeof(double));
    R[3][3] = 1.0;
    double nb = sqrt(bx * bx + by * by + bz * bz);
    if (nb == 0.0) {
        R[0][0] = R[1][1] = R[2][2] = 1.0;
        return;
    }
    double ux = bx / nb, uy = by / nb, uz = bz / nb;
    double theta = -OR_TWO_PI * OR_GAMMA_BAR * nb * dt;
    double c = cos(theta), s = sin(theta), v = 1.0 - c;
    R[0][0] = c + ux * ux * v;
    R[0][1] = -uz * s + ux * uy * v;
    R[0][2] = uy * s + ux * uz * v;
    R[1][0] = uz * s + ux * uy * v;
    R[1][1] = c + uy * uy * v;
    R[1][2] = -ux * s + uy * uz * v;
    R[2][0] = -uy * s + ux * uz * v;
    R[2][1] = ux * s + uy * uz * v;
    R[2][2] = c + uz * uz * v;
}

/* Eq. (A1): T2 decay of Mx, My; T1 recovery of Mz toward M0. */
static void relaxation_matrix(double dt, double t1, double t2, double D[4][4])
{
    memset(D, 0, 16 * sizeof(double));
    double e1 = exp(-dt / t1), e2 = exp(-dt / t2);
    D[0][0] = e2;
    D[1][1] = e2;
    D[2][2] = e1;
    D[2][3] = 1.0 - e1;
    D[3][3] = 1.0;
}

static void matmul4(double A[4][4], double B[4][4], double C[4][4])
{
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int l = 0; l < 4; ++l)
                s += A[i][l] * B[l][j];
            C[i][j] = s;
        }
}

static void matvec4(double A[4][4], const double v[4], double w[4])
{
    for (int i = 0; i < 4; ++i) {
        double s = 0.0;
        for (int l = 0; l < 4; ++l)
            s += A[i][l] * v[l];
        w[i] = s;
    }
}

/* Eq. (2): one raster step, U = D * R applied to the homogeneous vector.
 * D depends on dt, T1 and T2 only, so the caller builds it once per
 * isochromat. */
static void oracle_step(double M[4], double bx, double by, double bz, double dt, double D[4][4])
{
    double R[4][4], U[4][4], out[4];
    rotation_matrix(bx, by, bz, dt, R);
    matmul4(D, R, U);
    matvec4(U, M, out);
    memcpy(M, out, sizeof(out));
}

/* Eq. (4) and Eq. (5) over a block with B1 = 0. */
static void oracle_relax(double M[4], double tau, const double mom[3], double x, double y, double z,
                         double df, double t1, double t2)
{
    double cycles = OR_GAMMA_BAR * (mom[0] * x + mom[1] * y + mom[2] * z) + df * tau;
    double phase = OR_TWO_PI * (cycles - nearbyint(cycles));
    double e2 = exp(-tau / t2), e1 = exp(-tau / t1);
    double c = cos(phase), s = sin(phase);
    double mx = M[0], my = M[1];
    M[0] = e2 * (mx * c + my * s); /* (Mx + i My) * exp(-i phase) */
    M[1] = e2 * (my * c - mx * s);
    M[2] = M[3] + (M[2] - M[3]) * e1;
}

static int bad_time_constant(double t)
{
    return !(t > 0.0); /* rejects NaN, zero and negatives; +inf is allowed */
}

int oracle_simulate(int64_t K, const double *x, const double *y, const double *z, const double *t1,
                    const double *t2, const double *df, const double *m0, const double *m_init,
                    int64_t n_blocks, const int32_t *btype, const int64_t *step_offset,
                    const int64_t *n_steps, const int32_t *n_samples, const int64_t *sample_offset,
                    const double *tau, const double *moment, int64_t total_steps,
                    const double *rf_re, const double *rf_im, const double *gx, const double *gy,
                    const double *gz, int64_t total_samples, const int32_t *adc_idx, double dt,
                    int nthreads, double *m_out, double *sig_out)
{
    if (K < 0 || n_blocks < 0 || total_steps < 0 || total_samples < 0 || !(dt > 0.0))
        return OR_E_INVALID;
    if (K > 0 && (!x || !y || !z || !t1 || !t2 || !df || !m0 || !m_out))
        return OR_E_INVALID;
    if (total_samples > 0 && (!sig_out || !adc_idx))
        return OR_E_INVALID;
    for (int64_t b = 0; b < n_blocks; ++b) {
        if (btype[b] == OR_BLOCK_RELAX) {
            if (!(tau[b] >= 0.0))
                return OR_E_INVALID;
            continue;
        }
        if (btype[b] != OR_BLOCK_RF && btype[b] != OR_BLOCK_ADC)
            return OR_E_INVALID;
        if (n_steps[b] < 0 || step_offset[b] < 0 || step_offset[b] + n_steps[b] > total_steps)
            return OR_E_INVALID;
        if (n_samples[b] < 0 || sample_offset[b] < 0 || sample_offset[b] + n_samples[b] > total_samples)
            return OR_E_INVALID;
        if (btype[b] == OR_BLOCK_RF && n_samples[b] != 0)
            return OR_E_INVALID;
        for (int32_t n = 0; n < n_samples[b]; ++n) {
            int32_t s = adc_idx[sample_offset[b] + n];
            if (s < 0 || s > n_steps[b])
                return OR_E_INVALID;
            if (n > 0 && s < adc_idx[sample_offset[b] + n - 1])
                return OR_E_INVALID; /* samples must be in time order */
        }
    }
    for (int64_t k = 0; k < K; ++k)
        if (bad_time_constant(t1[k]) || bad_time_constant(t2[k]) || isnan(x[k]) || isnan(y[k]) ||
            isnan(z[k]) || isnan(df[k]) || isnan(m0[k]))
            return OR_E_INVALID;

    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
#endif
    double *part = NULL;
    if (total_samples > 0) {
        part = (double *)calloc((size_t)nt * 2 * (size_t)total_samples, sizeof(double));
        if (!part)
            return OR_E_NOMEM;
    }

#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = part ? part + (size_t)tid * 2 * (size_t)total_samples : NULL;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t k = 0; k < K; ++k) {
            double M[4];
            if (m_init) {
                M[0] = m_init[k];
                M[1] = m_init[K + k];
                M[2] = m_init[2 * K + k];
            } else {
                M[0] = 0.0;
                M[1] = 0.0;
                M[2] = m0[k];
            }
            M[3] = m0[k];
            double bz_off = df[k] / OR_GAMMA_BAR; /* tesla */
            double D[4][4];
            relaxation_matrix(dt, t1[k], t2[k], D);
            for (int64_t b = 0; b < n_blocks; ++b) {
                if (btype[b] == OR_BLOCK_RELAX) {
                    oracle_relax(M, tau[b], moment + 3 * b, x[k], y[k], z[k], df[k], t1[k], t2[k]);
                    continue;
                }
                int64_t s0 = step_offset[b], ns = n_steps[b];
                int64_t so = sample_offset[b];
                int32_t nsamp = n_samples[b], next = 0;
                for (int64_t j = 0; j <= ns; ++j) {
                    while (next < nsamp && adc_idx[so + next] == j) {
                        acc[2 * (so + next)] += M[0];
                        acc[2 * (so + next) + 1] += M[1];
                        ++next;
                    }
                    if (j == ns)
                        break;
                    int64_t s = s0 + j;
                    double bz = gx[s] * x[k] + gy[s] * y[k] + gz[s] * z[k] + bz_off;
                    oracle_step(M, rf_re[s], rf_im[s], bz, dt, D);
                }
            }
            m_out[k] = M[0];
            m_out[K + k] = M[1];
            m_out[2 * K + k] = M[2];
        }
    }

    if (total_samples > 0) {
        memset(sig_out, 0, 2 * (size_t)total_samples * sizeof(double));
        for (int t = 0; t < nt; ++t)
            for (int64_t i = 0; i < 2 * total_samples; ++i)
                sig_out[i] += part[(size_t)t * 2 * (size_t)total_samples + i];
        free(part);
    }
    return OR_OK;
}

/* Number of OpenMP threads an oracle call uses when nthreads <= 0. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
