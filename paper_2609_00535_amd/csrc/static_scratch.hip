// Device memory of the allocation-free batched step (slbm_batch_step_static): one
// file-scope array per GPU that holds the batch's launch tables, so that the step calls no
// device allocator.  The array's name is a host-side stand-in in host code; its device
// address is looked up once per device (with that device current) and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace slbm {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
}  // namespace

int static_scratch(void **ptr) {
    int dev = 0;
    int e = (int)hipGetDevice(&dev);
    if (e) return e;
    if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = (int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e) return e;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return 0;
}

}  // namespace slbm
