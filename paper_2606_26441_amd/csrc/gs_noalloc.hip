// Fixed scratch memory of the allocation-free search (gs_search_batch_noalloc):
// one device array per GPU, holding the search workspace (score rows, histograms,
// selection state, candidate buffers), for callers that cannot allocate device
// memory. Each device holds its own copy of the array until the process ends.
#include <mutex>

#include "gs_internal.h"

// The host-side name of this array is a stand-in, not a device address: host code
// uses only the address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[gs::kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace gs {

hipError_t scratch_address(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> l(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace gs
