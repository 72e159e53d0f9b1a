// noalloc.hip -- the argument staging of esk_render_batch_noalloc: a static
// device array instead of a caller workspace, for callers that cannot
// allocate.  The per-device set-up (esk_create on a device) resolves the
// array's device address once per device and allocates the pinned host
// staging and event that the entry point then reuses; the entry point
// itself allocates nothing.
#include <mutex>

#include "esk_internal.hpp"

namespace esk {

// Per-request render arguments of the last batched call on this device.
// Host code never names it directly: every use goes through the address
// returned by hipGetSymbolAddress below.
static __device__ __align__(256) RenderArgs scratch[kNoAllocBatchMax];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
NoAllocSlot g_slot[kMaxDevices];

}  // namespace

hipError_t noalloc_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    NoAllocSlot &s = g_slot[device];
    if (s.d_args) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    RenderArgs *host = nullptr;
    e = hipHostMalloc(reinterpret_cast<void **>(&host), sizeof(RenderArgs) * kNoAllocBatchMax);
    if (e != hipSuccess) return e;
    hipEvent_t done = nullptr;
    e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipHostFree(host);
        return e;
    }
    s.h_staging = host;
    s.done = done;
    s.recorded = false;
    s.d_args = static_cast<RenderArgs *>(ptr);   // published last: a set slot is complete
    return hipSuccess;
}

NoAllocSlot *noalloc_slot(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_slot[device].d_args ? &g_slot[device] : nullptr;
}

}  // namespace esk
