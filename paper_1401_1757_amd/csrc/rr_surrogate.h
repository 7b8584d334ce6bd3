// Learned reserve surrogate: internal interface between the context
// (rr_host.cpp) and the surrogate runtime (rr_surrogate.cpp).
#pragma once

namespace rr {

struct Surrogate;
void surrogate_destroy(Surrogate *s);

}  // namespace rr
