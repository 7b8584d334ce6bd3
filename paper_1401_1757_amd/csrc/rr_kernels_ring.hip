// Curve-ring instances of the reserve recurrence kernel (level single- and
// joint-life portfolios): the scenario discount factors of an item pass
// through a per-wavefront LDS ring instead of scalar loads.
#include "rr_recurrence.h"

namespace rr {

bool supported_ring(int K, int J)
{
    return (K == 16 && (J == 1 || J == 2)) || (K == 8 && J == 2);
}

hipError_t launch_recurrence_ring(int K, int J, const RecParams &p, int grid, size_t lds_bytes,
                                  hipStream_t stream)
{
    switch (J * 64 + K) {
    case 64 + 16: launch_kj_ring<16, 1>(p, grid, lds_bytes, stream); break;
    case 128 + 16: launch_kj_ring<16, 2>(p, grid, lds_bytes, stream); break;
    case 128 + 8: launch_kj_ring<8, 2>(p, grid, lds_bytes, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace rr
