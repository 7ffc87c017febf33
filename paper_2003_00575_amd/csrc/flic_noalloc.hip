// flic_noalloc.hip -- device scratch of the allocation-free entry point.
//
// flic_cluster_noalloc takes its scratch (masks, run roots, border slots,
// parent array) from the file-scope device array below instead of a
// context's hipMalloc'd ring.  Every device the library runs on holds its own
// copy of the array until the process ends.  In host code the array's name
// is only a host-side stand-in, so the kernels get the device address that
// hipGetSymbolAddress returns, fetched once per device with that device
// current and kept here.
#include <mutex>

#include "flic_internal.h"

namespace flic {
namespace {

__device__ __align__(256) char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace flic
