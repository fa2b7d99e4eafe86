// Allocation-free evaluation: qdvm_eval with its device scratch in a static
// array of this library instead of the plan's workspace (see qdvm.h).
#include <hip/hip_runtime.h>

#include <mutex>

#include "qdvm_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;   // 32 MiB per GPU

// One copy per GPU the library runs on, held until the process ends.  Host
// code never passes this name to a kernel: it stands for a host-side symbol,
// not a device address.  The device address of each GPU's copy comes from
// hipGetSymbolAddress (scratch_address below).
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

// Device address of the current GPU's scratch, looked up once per device with
// that device current.
qdvm_status scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return qdvm::record_error(QDVM_EDEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return qdvm::record_error(QDVM_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return qdvm::record_error(QDVM_EDEVICE, "hipGetSymbolAddress of the static scratch failed");
        g_addr[dev] = ptr;
    }
    *out = g_addr[dev];
    return QDVM_OK;
}

}  // namespace

extern "C" {

qdvm_status qdvm_eval_noalloc(qdvm_plan_t plan, int32_t batch, const float* f, float* q, const float* w, float dt,
                              hipStream_t stream)
{
    if (!plan) return qdvm::record_error(QDVM_EINVAL, "null plan");
    if (batch == 0) return QDVM_OK;
    void* ws = nullptr;
    const qdvm_status s = scratch_address(&ws);
    if (s != QDVM_OK) return s;
    return qdvm::eval_with_scratch(plan, batch, f, q, w, dt, stream, ws, kScratchBytes);
}

size_t qdvm_noalloc_scratch_bytes(void) { return kScratchBytes; }

}  // extern "C"
