// Allocation-free logB of stored 2F maps (tfstat_logB_noalloc).
//
// The reduction of a stored map (appendix A footnote: logB is the
// max-shifted log of the mean of exp(F) over the map) needs a workspace for
// its per-tile partials and per-map results.  tfstat_logB sub-allocates it
// from the context's arena and stages the results through pinned host
// memory; this entry point instead keeps the workspace in one file-scope
// device array per GPU and writes logB to device memory, so that a call
// allocates nothing and can sit inside HIP graph capture.
//
// The array's host-side name is not a device address.  Its address on each
// device is looked up once, with that device current, when a context is
// created on it (tfstat_ctx_create calls noalloc_setup), and only that
// address is handed to kernels.
#include "../../include/tfstat.h"
#include "tfstat_device.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace {

__device__ __align__(256) unsigned char scratch[TFSTAT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {nullptr};

}  // namespace

namespace tfs {

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_mu);
    if (g_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
    return hipSuccess;
}

void *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_mu);
    return g_ptr[device];
}

}  // namespace tfs
