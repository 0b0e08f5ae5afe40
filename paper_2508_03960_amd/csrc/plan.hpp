// Host-side planning of a simulation: subsequence classification (Sec. 2.1,
// 2.4, 3.1) and the schedule of device passes for both modes.  Pure C++; no
// HIP dependency, so it is unit-testable without a GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "gbloch.h"

namespace gbs {

// Gradient type of a with-RF / with-ADC subsequence (Sec. 2.4).
enum GradType { GT_X = 0, GT_Y = 1, GT_Z = 2, GT_NONE = 3, GT_MIXED = 4 };

// RfJob::axis of a no-grads transition composed per tissue group (key T1, T2,
// dB0; built with GBS_AX_N) and applied through the x-group rows.
constexpr int kTissueAxis = 3;
// RfJob::axis of a Gx+Gz transition composed per two-axis group (key x, z,
// T1, T2, dB0; built with GBS_AX_XZ), and PassOp::rf_axis of its rows.
constexpr int kPairAxis = 4;
constexpr int kPairRows = 3;

struct HostSeq {
    std::vector<gbs_block> blocks;
    std::vector<float> rf_re, rf_im, gx, gy, gz;
    std::vector<int32_t> adc_idx;
    double dt = 0.0;
    int64_t total_steps = 0, total_samples = 0, stepped_steps = 0;
};

struct BlockClass {
    bool has_b1 = false;   // any nonzero B1 sample in the block
    int gtype = GT_NONE;   // exact-zero test per axis over the whole block
    int axes_mask = 0;     // bit a: gradient a is nonzero somewhere in the block
    double moment[3] = {0, 0, 0};  // sum_j G_j dt over the block (FP64)
};

// A B1 = 0 closed-form map (Eq. 4, 5) over total duration tau with total
// gradient moment m.  All such maps commute, so consecutive ones add.
struct Map {
    double tau = 0.0;
    double m[3] = {0.0, 0.0, 0.0};
    bool any() const { return tau != 0.0 || m[0] != 0.0 || m[1] != 0.0 || m[2] != 0.0; }
    void add(double t, const double *mm) {
        tau += t;
        m[0] += mm[0];
        m[1] += mm[1];
        m[2] += mm[2];
    }
};

// One streaming pass over all isochromats in group-sorted order:
//   M <- [RF group transition] o [pre map] (M), written back if write_m;
//   then, if emit_axis >= 0, the group sums of emit-map(Mxy) for ADC job adc_job.
struct PassOp {
    bool has_pre = false;
    Map pre;
    int rf_axis = -1;  // -1: none
    int rf_id = -1;    // index into Plan::rf
    bool write_m = true;
    int emit_axis = -1;
    Map emit;
    int adc_job = -1;
};

// Per-isochromat stepping of steps [step_lo, step_hi) of a block, with the
// samples [sample_lo, sample_hi) of that block (the plain method, or the
// fallback for a subsequence the grouped method cannot classify).
struct StepOp {
    int64_t block = -1;  // -1: no steps (closed-form pre map only)
    bool has_pre = false;
    Map pre;
    int64_t step_lo = 0, step_hi = 0;
    int32_t sample_lo = 0, sample_hi = 0;
};

// One operation of the conventional accelerated method (Sec. 2.2), per
// isochromat, after the pending closed-form map `pre`:
//   kind 2: with-RF block through its combined transition T_k (Eq. 7), which
//           the first occurrence of the waveform composes and caches;
//   kind 3: samples [sample_lo, sample_hi) of a with-ADC block without RF,
//           evaluated directly from the state at the block start by Eq. (4),
//           (5), (6); the state itself is not written (the block's map joins
//           the pending one);
//   kind 4: the pending map alone (always the last operation: writes the output).
struct CachedOp {
    int64_t block = -1;
    bool has_pre = false;
    Map pre;
    int entry = -1;        // kind 2: cache entry, index into Plan::rf (axis -1)
    bool compose = false;  // kind 2: first occurrence of the waveform
    int32_t sample_lo = 0, sample_hi = 0;  // kind 3
};

struct Op {
    int kind = 0;  // 0 = pass, 1 = step, 2-4 = CachedOp kinds
    PassOp pass;
    StepOp step;
    CachedOp cached;
};

struct RfJob {  // one distinct combined transition (Eq. 7) per group of `axis` (or kTissueAxis)
    int axis;
    int64_t step_offset, n_steps;
};

struct AdcJob {  // one grouped with-ADC subsequence (Eq. 8-10)
    int axis;
    int64_t block;
};

struct Plan {
    std::vector<Op> ops;
    std::vector<RfJob> rf;
    std::vector<AdcJob> adc;
    bool final_pass = false;  // materialize the trailing map before output
    Map final_map;
    int64_t n_rf_grouped = 0, n_adc_grouped = 0, n_fallback = 0, n_b1zero = 0, n_relax = 0;
    int64_t n_passes = 0, n_emit_only = 0;
    int64_t n_rf_cached = 0, n_adc_direct = 0;  // plan_cached
};

// Largest number of ADC samples one stepping launch accumulates (LDS bound).
constexpr int32_t kMaxSamplesPerLaunch = 256;

int validate_sequence(const gbs_block *blocks, int64_t n_blocks, int64_t total_steps,
                      const int32_t *adc_idx, int64_t total_samples, double dt, std::string &err);
void copy_sequence(HostSeq &s, const gbs_block *blocks, int64_t n_blocks, const float *rf_re,
                   const float *rf_im, const float *gx, const float *gy, const float *gz,
                   int64_t total_steps, const int32_t *adc_idx, int64_t total_samples, double dt);
std::vector<BlockClass> classify(const HostSeq &s);
// max_samples: the most samples one stepping launch accumulates (kMaxSamplesPerLaunch
// divided by the receive coils, whose sums share the launch's LDS)
Plan plan_plain(const HostSeq &s, int32_t max_samples = kMaxSamplesPerLaunch);
Plan plan_grouped(const HostSeq &s, const std::vector<BlockClass> &cls, uint32_t axes_built,
                  int32_t max_samples = kMaxSamplesPerLaunch);
// Schedule of the conventional accelerated method with dynamic caching of
// per-isochromat transitions (Sec. 2.2).  Plan::rf lists the cache entries
// (axis -1: bit-identical B1 and all three gradients).
Plan plan_cached(const HostSeq &s, const std::vector<BlockClass> &cls, int32_t max_samples = kMaxSamplesPerLaunch);

}  // namespace gbs
