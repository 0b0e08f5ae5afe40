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
    float *mout_x, *mout_y, *mout_z;     // state out (may alias state in; null: not written)
    // FP64 state carried between launches of the FP64 stepper (null: unused);
    // when min64_x is set it replaces min_*
    const double *min64_x, *min64_y, *min64_z;
    double *mout64_x, *mout64_y, *mout64_z;
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

// ---- grouped sweep -------------------------------------------------------
// One grouped operation (Sec. 2.3) inside a sweep:
//   M <- T'_g o [remaining pre-map phases] (M), where T' is the group
//   transition with the tissue and own-axis part of the preceding B1 = 0 map
//   folded in; then, if emitting, the group sums of emit-map(Mxy) for one
//   with-ADC subsequence (Eq. 9).  An operation without a transition applies
//   its whole pre map per isochromat (kPreMz: with T1 recovery).
// y phases of consecutive emissions follow a recurrence when their
// coefficients step evenly (kYDirect starts it, kYSetR sets the step, kYStep
// advances it).  In a sweep without such recurrences the same per-isochromat
// factor holds a repeated y phase of the pre maps instead (kPreYSet evaluates
// it, kPreYHold reuses it).  Every wavefront reads the descriptor with scalar
// loads.
enum {
    kOpPre = 1,
    kOpRf = 2,
    kOpEmit = 4,
    kPreMz = 8,
    kYDirect = 16,
    kYStep = 32,
    kYSetR = 64,
    kPreYSet = 128,
    kPreYHold = 256
};
// An emission that starts a chain (kYDirect) also carries, in bits
// kChainShift.., the number of kYStep emissions that follow it (at most 15).
enum { kChainShift = 12, kChainMask = 15 };
struct SweepOp {
    int32_t flags;
    int32_t rf_axis;
    int32_t emit_axis;
    int32_t gsum_stride;     // groups of the emission axis: coil p sums at gsum + p * gsum_stride
    const float4 *pre_xtab;  // per x-group (Re a, Im a, E1, 0); null: no x factor
    float4 *part;            // kPartials: this x-emission's per-wavefront sums, one float4 per
                             // wavefront of 512 slots (fast and emission-only sweeps)
    const float2 *pre_ztab;  // per z-group phase; null: none
    double pre_cy, pre_cz;   // direct y / z phase coefficients (cycles per metre); 0: none
    const float4 *ttab;      // 3 float4 rows (A_r0, A_r1, A_r2, b_r) per group of rf_axis
    const float4 *emit_xtab; // per x-group: decay, off-resonance and x phase
    const float2 *emit_ztab; // per z-group phase; null: none
    double emit_cy;          // y phase coefficient (cycles per metre)
    double emit_dcy;         // recurrence step of emit_cy (kYSetR)
    double emit_cz;          // direct z phase coefficient (no z groups)
    double2 *gsum;
};

// Per-isochromat arrays a sweep reads.
enum { kNeedMz = 1, kNeedGx = 2, kNeedGy = 4, kNeedGz = 8, kNeedY = 16, kNeedZ = 32, kNeedRun = 64 };
// Set in SweepArgs::need of a segment whose every op only emits (no pre map,
// no transition): it runs in the emission-only sweep.  kEmitTail: the last
// op of such a segment is a B1 = 0 map without transition or emission (the
// closed form that ends the sequence), applied after the emissions.
enum { kEmitOnly = 128, kEmitTail = 256 };
// kEmitHead: the first SweepArgs::n_head ops of such a segment are general
// ops (pre map, x- or z-group transition, emission without a stepped y phase)
// applied to the state before the emissions.
enum { kEmitHead = 2048 };
// kPartials: the x-group sums of the segment's emissions go to per-wavefront
// partial sums (SweepOp::part) instead of memory-side atomics: lane 63 of a
// wavefront of 512 isochromats (8 per thread) stores (sum of its first
// key, sum of the other key) as one float4; k_part_reduce then adds, per
// group, the entries of the wavefronts that span it.  A wavefront with three
// or more keys stores zeros and adds its sums with atomics.
enum { kPartials = 1024 };
// Run the segment in the general sweep, which keeps M itself in registers
// (the fast sweeps hold M / M0): set for a run whose initial state gives an
// isochromat with M0 = 0 a nonzero magnetization.
enum { kForceGeneral = 512 };

// A sweep applies ops[0 .. n_ops) in order to every isochromat while its
// state stays in registers: one read and at most one write of M per launch.
// The layout pads runs of equal (x-group, z-group) to multiples of 8, so the
// 4 or 8 consecutive isochromats of a thread share their x- and z-groups.
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
    // Final sweep of a run: when set, the state is written here as
    // (mx, my, mz, 0) per layout slot instead of into mx / my / mz, so that
    // the copy into the caller's order reads one 16-byte row per isochromat.
    float4 *m_final;
    // First sweep of a run from the default state (0, 0, M0): nothing is read
    // from mx / my / mz.
    int32_t fresh;
    int32_t n_head;  // kEmitHead
    // Receive-coil sensitivities (Eq. 6 with S(k, p)), or null for one coil of
    // unit sensitivity: planes re, im of coil 0, re, im of coil 1, ... of
    // coil_plane float4 words each in layout order.  Every emission weights
    // its members by S(k, p) before the group sums of coil p (general sweep).
    const float4 *coil;
    int32_t n_coils;
    int64_t coil_plane;
    // Two-axis group (run of equal x- and z-group) of every 4-slot quad, for
    // operations whose transition rows are per such group (rf_axis 3; general sweep)
    const int32_t *run_of4;
};

// One emission of a kPartials segment: gsum[g] += the entries of part that
// belong to group g.
struct PartJob {
    const float4 *part;
    double2 *gsum;
};
hipError_t launch_part_reduce(const PartJob *jobs, int n_jobs, int64_t n_groups, const int32_t *xstart,
                              hipStream_t st);
// xstart[g] <- first slot of x-group g in the layout (slots [0, n)), xstart[G] <- n
hipError_t launch_group_starts(int64_t n, const int32_t *gid_x, int64_t n_groups, int32_t *xstart, hipStream_t st);
// slots of the layout one wavefront of the emission-only sweep covers
constexpr int kPartSlots = 512;

// ---- tables ---------------------------------------------------------------
struct TabJob {
    int32_t kind;  // 0: x-group decay, off-resonance, x phase, E1 (float4); 1: z-group phase (float2);
                   // 2: x-group x phase only (float4, E1 = 1)
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
    double *out;         // 12 doubles (A row-major, b) per group
};

// T' = T o P for one operation: P is the tissue part (decay, off-resonance,
// T1 recovery) and the own-axis phase of its pre map (identity if none).
struct FoldJob {
    int32_t axis;
    int32_t has_pre;
    int64_t n_groups;
    const double *t64;
    const float4 *gtab;
    double tau;
    double cyc;  // gamma_bar * moment along `axis`
    float4 *out;
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
hipError_t launch_plain(const PlainArgs &a, bool has_b1, int grid, hipStream_t st);
hipError_t launch_plain_finalize(const double2 *partial, int nblk, int n_samples, double *sig,
                                 hipStream_t st);
int plain_grid(int64_t K);

hipError_t launch_sweep(const SweepArgs &a, hipStream_t st);
hipError_t launch_tables(const TabJob *jobs, int n_jobs, int max_n, const float4 *gtab_x,
                         const float4 *gtab_z, hipStream_t st);
hipError_t launch_compose(const RfJobDev *jobs, int n_jobs, int64_t max_groups, double dt,
                          hipStream_t st);
hipError_t launch_fold(const FoldJob *jobs, int n_jobs, int64_t max_groups, hipStream_t st);
hipError_t launch_adc_eval(const AdcJobDev *jobs, int n_jobs, int max_groups, int max_samples,
                           double *sig, hipStream_t st);
hipError_t launch_fill_f64(double *p, int64_t n, hipStream_t st);
hipError_t launch_init_state(int64_t K, int64_t Kpad, const int32_t *perm, const float *mi_x,
                             const float *mi_y, const float *mi_z, const float *m0i, float *mx,
                             float *my, float *mz, hipStream_t st);
hipError_t launch_gather_state(int64_t K, const int32_t *inv, const float *mx, const float *my, const float *mz,
                               float *ox, float *oy, float *oz, hipStream_t st);
hipError_t launch_gather_state4(int64_t K, const int32_t *inv, const float4 *m4, float *ox, float *oy, float *oz,
                                hipStream_t st);
// *flag <- 1 if some isochromat has M0 = 0 and a nonzero initial state (*flag
// is not cleared)
hipError_t launch_check_zero_m0(int64_t K, const float *m0, const float *mx, const float *my, const float *mz,
                                int *flag, hipStream_t st);

// ---- grouping ---------------------------------------------------------------
hipError_t launch_validate_phantom(int64_t K, const PhantomPtrs &ph, int *bad, hipStream_t st);

}  // namespace gbs
