// Hooks between the context code (api.cpp) and the static-scratch entry
// point (noalloc.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "gbloch.h"

namespace gbs {

// Looks up this device's static scratch array (call with `device` current).
hipError_t noalloc_setup(int device);
// The context's device, and its error reporting.
int ctx_device(const gbs_ctx *ctx);
int ctx_fail(gbs_ctx *ctx, int code, const char *msg);

}  // namespace gbs
