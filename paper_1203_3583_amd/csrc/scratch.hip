// A fixed device scratch array for callers that cannot allocate device memory.
//
// The array is a file-scope device variable: every GPU the library runs on holds
// its own copy, from the code object's load until the process ends.  In host code
// its name is only a stand-in; the device address is looked up once per device
// with hipGetSymbolAddress (with that device current) and kept, and only that
// address is ever handed to kernels or copies.
#include <mutex>

#include "asf_internal.h"

namespace asf {
namespace {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
void *g_addr[kMaxDevices];   // the array's address on each device, once looked up
std::mutex g_lock;

}  // namespace

hipError_t static_scratch(void **out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> hold(g_lock);
    if (!g_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return hipSuccess;
}

}  // namespace asf
