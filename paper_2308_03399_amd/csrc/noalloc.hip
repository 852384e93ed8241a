// Library-owned device buffer of the no-allocation entry point
// (sv_run_circuit_noalloc): callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc) run the executor on this file-scope array instead of an arena
// they attach. Every GPU the library runs on holds its own copy, at its own
// address, from module load until the process ends.
//
// In host code the array's name is only a stand-in for the symbol, not a
// device address: the address of each device's copy comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that pointer is ever passed to kernels or copies.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

namespace {

constexpr uint64_t kScratchBytes = 64ull << 20;  // the stated maximum (SV_NOALLOC_MAX_BYTES)
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices];

}  // namespace

extern "C" {

// Device address of this device's scratch array and its size. The first
// call on a device resolves the address (with that device current) and
// keeps it; later calls return the kept pointer.
hipError_t svb_noalloc_scratch(void **ptr, uint64_t *bytes)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    *bytes = kScratchBytes;
    return hipSuccess;
}

}  // extern "C"
