// fft_execute_scratch: fft_execute without any device allocation.  A two-pass
// plan's intermediate goes through `scratch`, a fixed device array of the
// library, instead of the plan's workspace; single-pass plans use no scratch.
#include "dsfft.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "plan.hpp"

namespace dsfft {
namespace {

static_assert(FFT_SCRATCH_BYTES % 256 == 0, "whole 256-byte blocks");

// One copy per GPU, held from the library's load until the process ends.  In
// host code this name is only the runtime's handle for the variable; its device
// address comes from hipGetSymbolAddress below.
__device__ __align__(256) unsigned char scratch[FFT_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];   // device address of `scratch`, per device

// The device address of `scratch` on the current device, looked up on the
// first call made with that device current.
int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return set_error(FFT_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return set_error(FFT_EHIP, "hipGetSymbolAddress(scratch) gave a null address");
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return FFT_OK;
}

}  // namespace
}  // namespace dsfft

using namespace dsfft;

extern "C" int fft_execute_scratch(fft_plan* plan, const void* in, void* out, void* stream) {
    int rc = check_execute_args(plan, in, out);
    if (rc != FFT_OK) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev != plan->device) return set_error(FFT_EINVAL, "the plan's device is not the current device");
    if (!plan->k2) return launch_plan_ws(plan, in, out, (hipStream_t)stream, nullptr, plan->batch);
    // two-pass: as many transforms per chunk as the scratch holds
    const size_t per = (size_t)plan->n * work_elem_bytes(plan->dtype);
    if (per > FFT_SCRATCH_BYTES)
        return set_error(FFT_EINVAL, "one transform's intermediate exceeds FFT_SCRATCH_BYTES");
    void* ws = nullptr;
    rc = scratch_address(dev, &ws);
    if (rc != FFT_OK) return rc;
    const int64_t chunk = std::min<int64_t>(plan->batch, (int64_t)(FFT_SCRATCH_BYTES / per));
    return launch_plan_ws(plan, in, out, (hipStream_t)stream, ws, chunk);
}
