// Device scratch of the entry point that allocates nothing
// (ocr_reuse_ao_noalloc): a file-scope array that every device the library
// runs on holds from the code object's load until the process ends, and its
// address on each device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "api_internal.hpp"

namespace ocr {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// The array's device address on the current device.  hipGetSymbolAddress is
// called once per device, with that device current; its address is kept and
// used for every later call on that device (in host code the array's name is
// no device address).  Returns the HIP error of the lookup, if any.
hipError_t scratch_address(void **ptr) {
    static std::mutex mu;
    static void *addr[kMaxScratchDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace ocr
