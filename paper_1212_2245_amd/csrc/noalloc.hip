// Library-owned scratch for the entry point that allocates nothing
// (deblur_rrrl_iterate_noalloc): a file-scope device array that every GPU the
// library runs on holds from module load until the process ends.
//
// In host code the array's name is only a host-side stand-in for the symbol;
// its device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and kept, and only that address is ever handed
// to kernels or copies.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>
#include <vector>

#include "launch.hpp"

namespace deblur {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// Device address of this device's copy of `scratch`, or nullptr if the lookup
// failed (the status is returned in *err).  Thread-safe; the lookup runs once
// per device.
void* noalloc_scratch(hipError_t* err)
{
    static std::mutex mu;
    static std::vector<void*> ptrs;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if ((int)ptrs.size() <= dev) ptrs.resize(dev + 1, nullptr);
    if (!ptrs[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        ptrs[dev] = ptr;
    }
    *err = hipSuccess;
    return ptrs[dev];
}

}  // namespace deblur
