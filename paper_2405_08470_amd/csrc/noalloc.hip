// The fixed device buffer of spt_mttkrp_noalloc: the partial sums of rows
// split across partitions (the only scratch the elementwise kernel and the
// fixup use), for callers that cannot allocate device memory.  The array
// exists once per device for the life of the process; its device address is
// taken with hipGetSymbolAddress once per device, with that device current,
// and only that address is handed to kernels (the array's name is not a
// device address in host code).
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace spt {

namespace {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mutex;
void* g_ptr[64] = {};

}  // namespace

hipError_t noalloc_scratch(void** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return hipSuccess;
}

}  // namespace spt
