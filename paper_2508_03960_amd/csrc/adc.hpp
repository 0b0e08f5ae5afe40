// ADC samples from group sums (Eq. 8 with Eq. 10) for readouts whose sample
// times and gradient moments are arithmetic in the sample index.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace gbs {

// Sample n of the block is taken at tau0 + n dtau after the block start, with
// gamma_bar * (gradient moment since the block start) = cyc0 + n dcyc.
struct AdcLinJob {
    int32_t n_samples;
    int32_t n_groups;
    const double2 *gsum;
    const float4 *gtab;  // (coord, T1, T2, df) per group
    double tau0, dtau;
    double cyc0, dcyc;
    int64_t sig_offset;
};

hipError_t launch_adc_lin(const AdcLinJob *jobs, int n_jobs, int max_groups, double *sig, hipStream_t st);

}  // namespace gbs
