// Device scratch of the entry points that allocate nothing
// (ci_hamiltonian_vjp_noalloc): one file-scope device array per GPU, held
// from the first call on that GPU until the process ends.  Host code never
// passes the array's name to a kernel (in host code it is a stand-in, not a
// device address): the device address is read once per device with
// hipGetSymbolAddress, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ci_internal.h"

namespace ci {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per device

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Device address of the scratch array on the current device (hipSuccess and
// *p set), cached per device after the first call.
hipError_t noalloc_scratch(void** p)
{
    constexpr int kDevs = 64;
    static std::mutex mu;
    static void* addr[kDevs] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kDevs) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        addr[dev] = ptr;
    }
    *p = addr[dev];
    return hipSuccess;
}

}  // namespace ci
