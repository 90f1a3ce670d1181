// fwi_static.hip -- the device array behind fwi_gradient_noalloc.
//
// `scratch` is a file-scope device array of FWI_NOALLOC_MAX_BYTES that serves as the
// workspace of the allocation-free gradient.  Every GPU the library runs on holds its own
// copy from the loading of the library's code object until the process ends.  In host
// code the array's name is only a stand-in: the device address of the current GPU's copy
// comes from hipGetSymbolAddress, taken once per device with that device current, and
// that address is what the kernels receive.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/fwi.h"

namespace fwi {

static __device__ __align__(256) uint8_t scratch[FWI_NOALLOC_MAX_BYTES];

// Device address of the current device's `scratch` (looked up on the first call made
// with that device current, then cached per device).
hipError_t noalloc_scratch(void **ptr, size_t *bytes)
{
    static std::mutex m;
    static std::vector<void *> addr;  // per device ordinal; nullptr until looked up
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(m);
    if ((size_t)dev >= addr.size()) addr.resize((size_t)dev + 1, nullptr);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = FWI_NOALLOC_MAX_BYTES;
    return hipSuccess;
}

}  // namespace fwi
