// Fixed device scratch for the entry point that allocates nothing
// (lp_spmv_noalloc): the partial vectors of the column-sliced product, the
// chunk sums of its long rows and, in mixed precision, the FP32 copies of
// its input and output live in one file-scope device array instead of
// memory the library allocates.  Every GPU the library runs on holds its own
// copy of the array until the process ends.
#include "internal.h"

#include <mutex>

namespace pdlp {
constexpr int kMaxDevices = 64;
}

// The name is only meaningful in device code: host code takes the array's
// per-device address from noalloc_scratch() and never uses `scratch` itself.
static __device__ __align__(256) unsigned char scratch[pdlp::kNoallocScratchBytes];

namespace pdlp {

namespace {
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};
}  // namespace

// Address of the array on the current device, looked up once per device
// (with that device current) and kept.  lp_load calls it, so the lookup
// happens at set-up and never during a later captured call.
hipError_t noalloc_scratch(void **ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[dev] = p;
    }
    *ptr = g_addr[dev];
    return hipSuccess;
}

}  // namespace pdlp
