// mxfft_static.hip -- the forward transform with its workspace in a static
// device array (mxfft_forward_static): no device allocation at any call.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "mxfft.h"
#include "mxfft_internal.hpp"

// The shared workspace.  In host code this name stands for the array but is
// not its device address: only the address looked up below reaches kernels.
static __device__ __align__(256) uint8_t scratch[MXFFT_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];   // device address of `scratch` per device, once known

// Address of the current device's copy of `scratch`, looked up on the first
// call on that device (with the device current) and kept.
mxfft_status scratch_address(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return MXFFT_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MXFFT_EHIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return MXFFT_OK;
}

}  // namespace

extern "C" mxfft_status mxfft_forward_static(mxfft_plan_t plan, const void* in, void* out, int32_t batch,
                                             int32_t* k_out, void* stream)
{
    if (!plan || !in || !out || batch < 0 || batch > 65535) return MXFFT_EINVAL;
    if (batch == 0) return MXFFT_OK;
    size_t bytes = 0;
    mxk::plan_workspace_layout(plan, batch, nullptr, nullptr, &bytes);
    if (bytes > (size_t)MXFFT_STATIC_SCRATCH_BYTES) return MXFFT_EBUDGET;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return MXFFT_EHIP;
    if (dev != mxk::plan_device(plan)) return MXFFT_EINVAL;
    void* base = nullptr;
    const mxfft_status st = scratch_address(dev, &base);
    if (st != MXFFT_OK) return st;
    mxk::Workspace w;
    mxk::plan_workspace_layout(plan, batch, (char*)base, &w, &bytes);
    return mxk::plan_forward_ws(plan, w, in, out, batch, k_out, stream);
}
