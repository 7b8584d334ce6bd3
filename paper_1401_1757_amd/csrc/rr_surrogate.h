// Learned reserve surrogate: internal interface between the C ABI (rr_host.cpp)
// and the MLP kernels (rr_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

struct rr_ctx;

namespace rr {

struct Surrogate;
void surrogate_destroy(Surrogate *s);

// Accessors into the context (rr_host.cpp).
int ctx_device(rr_ctx *c);
hipStream_t ctx_stream(rr_ctx *c);
int ctx_fail(rr_ctx *c, int code, const char *msg);
Surrogate *&ctx_surrogate(rr_ctx *c);

}  // namespace rr
