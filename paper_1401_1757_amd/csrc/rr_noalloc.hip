// Static device scratch of rr_reserve_recurrence_noalloc: a file-scope
// device array that every context on a GPU shares, so that the entry point
// needs no device allocation.  Host code never passes the array's name to a
// kernel or a copy (on the host it is only a stand-in for the symbol); it
// uses the device address that hipGetSymbolAddress returns for the current
// device, looked up once per device and kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rr_internal.h"

namespace rr {

namespace {

__device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int MAX_DEVICES = 64;
std::mutex g_mutex;
void *g_ptr[MAX_DEVICES] = {};

}  // namespace

// The device address of the scratch array on `device`, which must be the
// current device.  The first call on a device looks it up; later calls return
// the kept address.
hipError_t noalloc_scratch(int device, void **ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = p;
    }
    *ptr = g_ptr[device];
    return hipSuccess;
}

}  // namespace rr
