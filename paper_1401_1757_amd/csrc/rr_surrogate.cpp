// Placeholder surrogate entry points (replaced by the MLP implementation).
#include "rr.h"
#include "rr_surrogate.h"

namespace rr {
struct Surrogate {};
void surrogate_destroy(Surrogate *s) { delete s; }
}  // namespace rr

extern "C" int rr_surrogate_train(rr_ctx *c, const rr_train_cfg *, rr_train_report *)
{
    return c ? rr::ctx_fail(c, RR_ESTATE, "surrogate not available") : RR_EINVAL;
}
extern "C" int rr_surrogate_get_weights(rr_ctx *c, void *, size_t, size_t *)
{
    return c ? rr::ctx_fail(c, RR_ESTATE, "surrogate not available") : RR_EINVAL;
}
extern "C" int rr_surrogate_set_weights(rr_ctx *c, const void *, size_t)
{
    return c ? rr::ctx_fail(c, RR_ESTATE, "surrogate not available") : RR_EINVAL;
}
extern "C" int rr_surrogate_infer(rr_ctx *c, const rr_run *, const rr_outputs *, rr_infer_report *)
{
    return c ? rr::ctx_fail(c, RR_ESTATE, "surrogate not available") : RR_EINVAL;
}
