// Kernel argument blocks and host-side launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbs {

// One raster step of the sequence as the kernels read it (32 bytes, so a
// wave-uniform step is one scalar load).  b1sq = |B1|^2.
struct StepW {
    float b1r, b1i, b1sq, gx, gy, gz, pad0, pad1;
};

struct PhantomPtrs {
    const float *x, *y, *z, *t1, *t2, *df, *m0;
};

// ---- plain per-isochromat stepping --------------------------------------
struct PlainArgs {
    int64_t K;
    PhantomPtrs ph;
    const float *min_x, *min_y, *min_z;  // state in; null: (0, 0, M0)
    float *mout_x, *mout_y, *mout_z;     // state out (may alias state in)
    const StepW *wave;                   // first raster step of this launch
    int32_t n_steps;
    const int32_t *sidx;  // sample boundaries, counted from the block start
    int32_t step_base;    // block-relative index of this launch's first step
    int32_t n_samples;
    double2 *partial;     // [gridDim.x][n_samples] per-workgroup sums
    int32_t has_pre;      // closed-form map applied before the steps
    double pre_tau;
    double pre_cyc[3];    // gamma_bar * moment (cycles per metre)
    double dt;
    double gdt;           // gamma * dt (rad / T)
};

// ---- grouped streaming pass ---------------------------------------------
struct MapTabs {
    const float4 *xtab;  // per x-group: (Re a, Im a, E1, 0)
    const float2 *ztab;  // per z-group phase factor; null -> direct z phase via cz
    double cy;           // gamma_bar * m_y; 0 -> no y phase
    double cz;           // gamma_bar * m_z for the direct z phase; 0 -> none
};

// One grouped operation (Sec. 2.3) inside a sweep:
//   M <- [RF group transition] o [pre map] (M); then, if emitting, the group
//   sums of emit-map(Mxy) for one with-ADC subsequence (Eq. 9).
// Read by every wavefront with scalar loads.
enum { kOpPre = 1, kOpRf = 2, kOpEmit = 4 };
struct SweepOp {
    int32_t flags;
    int32_t rf_axis;
    int32_t emit_axis;
    int32_t pad;
    MapTabs pre;
    const float4 *ttab;  // 3 float4 rows (A_r0, A_r1, A_r2, b_r) per group
    MapTabs emit;
    double2 *gsum;
};

// Per-isochromat arrays a sweep reads.
enum { kNeedMz = 1, kNeedGx = 2, kNeedGy = 4, kNeedGz = 8, kNeedY = 16, kNeedZ = 32 };

// A sweep applies ops[0 .. n_ops) in order to every isochromat while its
// state stays in registers: one read and at most one write of M per launch.
struct SweepArgs {
    int64_t n4;  // number of 4-isochromat chunks
    float4 *mx, *my, *mz;
    const float4 *m0;
    const int4 *gid_x, *gid_y, *gid_z;
    const float4 *yv, *zv;
    const SweepOp *ops;
    int32_t n_ops;
    int32_t need;
    int32_t write_m;
};

// ---- tables ---------------------------------------------------------------
struct TabJob {
    int32_t kind;  // 0: x-group map factor (float4), 1: z-group phase (float2)
    int32_t n;     // groups
    double tau;    // duration (kind 0)
    double cyc;    // gamma_bar * moment along the table's axis
    void *out;
};

struct RfJobDev {
    int32_t axis;
    int32_t n_steps;
    int64_t n_groups;
    const StepW *wave;
    const float4 *gtab;  // (coord, T1, T2, df) per group
    float4 *out;         // 3 float4 per group
};

struct AdcJobDev {
    int32_t n_samples;
    int32_t n_groups;
    const double2 *gsum;
    const float4 *gtab;
    const double2 *samp;  // (tau_n, gamma_bar * m_n) per sample, from the block start
    int64_t sig_offset;   // first output sample of this block
};

// ---- launchers (all asynchronous on `st`) -----------------------------------
hipError_t launch_plain(const PlainArgs &a, bool has_b1, bool fp32, int grid, hipStream_t st);
hipError_t launch_plain_finalize(const double2 *partial, int nblk, int n_samples, double *sig,
                                 hipStream_t st);
int plain_grid(int64_t K);

hipError_t launch_sweep(const SweepArgs &a, hipStream_t st);
hipError_t launch_tables(const TabJob *jobs, int n_jobs, int max_n, const float4 *gtab_x,
                         const float4 *gtab_z, hipStream_t st);
hipError_t launch_compose(const RfJobDev *jobs, int n_jobs, int64_t max_groups, double dt,
                          hipStream_t st);
hipError_t launch_adc_eval(const AdcJobDev *jobs, int n_jobs, int max_groups, int max_samples,
                           double *sig, hipStream_t st);
hipError_t launch_fill_f64(double *p, int64_t n, hipStream_t st);
hipError_t launch_init_state(int64_t K, int64_t Kpad, const int32_t *perm, const float *mi_x,
                             const float *mi_y, const float *mi_z, const float *m0i, float *mx,
                             float *my, float *mz, hipStream_t st);
hipError_t launch_scatter_state(int64_t K, const int32_t *perm, const float *mx, const float *my,
                                const float *mz, float *ox, float *oy, float *oz, hipStream_t st);

// ---- grouping ---------------------------------------------------------------
hipError_t launch_validate_phantom(int64_t K, const PhantomPtrs &ph, int *bad, hipStream_t st);

}  // namespace gbs
