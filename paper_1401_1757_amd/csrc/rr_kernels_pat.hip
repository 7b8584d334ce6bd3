// Instances of the reserve recurrence kernel with the payment-pattern paths
// (escalating and annually paid annuities), launched for portfolios that
// hold such policies.
#include "rr_recurrence.h"

namespace rr {

hipError_t launch_recurrence_pat(int K, int J, const RecParams &p, int grid, size_t lds_bytes,
                                 hipStream_t stream)
{
    return launch_switch<true>(K, J, p, grid, lds_bytes, stream);
}

}  // namespace rr
