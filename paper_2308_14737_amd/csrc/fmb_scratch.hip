// fmb_scratch.hip -- the device workspace of fmb_backward_noalloc: one fixed array per device,
// so that the call allocates nothing.  Its device address is looked up once per device (with
// that device current) and kept; host code never passes the array's name to a kernel, only that
// address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fmb.h"

namespace fmb {

constexpr size_t kScratchBytes = FMB_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

size_t scratch_bytes() { return kScratchBytes; }

// Device address of `scratch` on the current device.
hipError_t scratch_base(void **out)
{
    static std::mutex mu;
    static void *base[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!base[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        base[dev] = p;
    }
    *out = base[dev];
    return hipSuccess;
}

}  // namespace fmb
