// Fixed device scratch of vbd_step_static: the per-step state buffers of a
// forward step (iterate, x^t, y, Chebyshev history, contact flags) in a
// file-scope device array instead of the bound workspace, so that step
// allocates nothing.
//
// The array's name is a host-side stand-in in host code: kernels receive the
// device address that hipGetSymbolAddress returns, looked up once per device
// (with that device current) and kept here.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "vbd_static.h"

namespace vbd {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(int device, void **ptr)
{
    static std::mutex mu;
    static std::vector<void *> per_device;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) return hipErrorInvalidDevice;
    if ((size_t)device >= per_device.size()) per_device.resize((size_t)device + 1, nullptr);
    if (!per_device[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the caller makes it current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        per_device[device] = p;
    }
    *ptr = per_device[device];
    return hipSuccess;
}

}  // namespace vbd
