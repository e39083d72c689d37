// Allocation-free anneal: the same sweeps as nmc_anneal, with the call's
// acceptance-threshold tables staged in a fixed device array of the library
// instead of a buffer it allocates.  For callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/nmc.h"
#include "nmc_internal.h"

// Largest threshold upload of one call (tables plus, for a host profile, the
// class array).  Every device the library runs on holds one copy until the
// process ends.
constexpr size_t kScratchBytes = (size_t)16 << 20;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
// device address of `scratch` on each device, looked up once per device (the
// host-side symbol is not a device address and is never passed to a kernel)
uint8_t *g_scratch_ptr[kMaxDevices] = {};

int scratch_on_current_device(uint8_t **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return nmc::set_last_error(NMC_ERR_DEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices)
        return nmc::set_last_error(NMC_ERR_DEVICE, "device index outside the library's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return nmc::set_last_error(NMC_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed");
        g_scratch_ptr[dev] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return NMC_OK;
}

}  // namespace

extern "C" {

int nmc_anneal_noalloc(nmc_replicas *rep, const double *beta, int32_t n_classes, int32_t n_sweeps, int32_t profile,
                       const uint8_t *class_of, int64_t target, void *stream) {
    uint8_t *ptr = nullptr;
    const int rc = scratch_on_current_device(&ptr);
    if (rc != NMC_OK)
        return rc;
    return nmc::anneal_into(rep, beta, n_classes, n_sweeps, profile, class_of, target, stream, ptr, kScratchBytes);
}

size_t nmc_anneal_noalloc_capacity(void) { return kScratchBytes; }

}  // extern "C"
