// gbs_simulate_static: gbs_simulate with its workspace taken from a static
// device array, for callers that cannot allocate device memory.
//
// `scratch` is a file-scope device array of kStaticScratchBytes; every device
// the library runs on holds its own copy from module load until the process
// ends.  In host code the array's name is only a stand-in for the symbol, so
// its device address is looked up once per device (noalloc_setup, called by
// gbs_create with that device current) and kept in scratch_ptr[device]; only
// that address is ever passed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "gbloch.h"
#include "noalloc.hpp"

namespace {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;  // GBS_STATIC_WORKSPACE_BYTES
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

}  // namespace

static_assert(kStaticScratchBytes == GBS_STATIC_WORKSPACE_BYTES, "header and library disagree on the size");

namespace gbs {

// Device address of this device's scratch array; called with `device` current.
hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_ptr[device] = p;
    return hipSuccess;
}

}  // namespace gbs

extern "C" int gbs_simulate_static(gbs_ctx *ctx, int mode, uint32_t flags, const float *m_init, float *m_out,
                                   double *sig_out, gbs_stats *stats) {
    if (!ctx) return GBS_E_INVALID;
    const int dev = gbs::ctx_device(ctx);
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(scratch_mu);
        ws = dev >= 0 && dev < kMaxDevices ? scratch_ptr[dev] : nullptr;
    }
    if (!ws) return gbs::ctx_fail(ctx, GBS_E_HIP, "static scratch of this device was not set up");
    size_t need = 0;
    if (int rc = gbs_workspace_size(ctx, mode, &need)) return rc;
    if (need > kStaticScratchBytes) {
        const std::string msg = "this call needs " + std::to_string(need) + " bytes of workspace; the static scratch "
                                "holds " + std::to_string(kStaticScratchBytes) + " (use gbs_simulate)";
        return gbs::ctx_fail(ctx, GBS_E_WORKSPACE, msg.c_str());
    }
    return gbs_simulate(ctx, mode, flags, ws, kStaticScratchBytes, m_init, m_out, sig_out, stats);
}
