// Fixed device scratch for the allocation-free entry point (nufft3_exec_noalloc):
// one file-scope array per device, found once per device with
// hipGetSymbolAddress and handed out by a bump arena (plan.h, Arena).
#include <mutex>

#include "noalloc.h"

namespace nufft {

static __device__ __align__(256) unsigned char scratch[NUFFT_NOALLOC_BYTES];

static std::mutex scratch_mu;
static void *scratch_dev[NUFFT_NOALLOC_MAX_DEVICES];

// The current device's copy of the array.  In host code `scratch` names a
// host-side stand-in, not device memory: only the address obtained here may
// be passed to kernels or copies.
hipError_t noalloc_scratch(void **ptr, size_t *bytes)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NUFFT_NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_dev[dev] = p;
    }
    *ptr = scratch_dev[dev];
    *bytes = NUFFT_NOALLOC_BYTES;
    return hipSuccess;
}

}  // namespace nufft
