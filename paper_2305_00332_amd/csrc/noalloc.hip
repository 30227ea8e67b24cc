// mmlttb_minmaxlttb_noalloc: MinMaxLTTB with its workspace in a fixed array of
// device memory that the library holds, for callers that cannot allocate
// (code under graph capture, tight serving loops, harnesses that forbid
// hipMalloc). The call itself allocates nothing and frees nothing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "errors.hpp"
#include "libmmlttb.h"

// The workspace of every mmlttb_minmaxlttb_noalloc call on a device. Each
// device holds its own copy, at its own address, until the process ends. In
// host code this name stands for the host-side shadow of the array, not for
// device memory: only the address looked up below may reach a kernel.
static __device__ __align__(256) unsigned char scratch[MMLTTB_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_scratch[kMaxDevices]; // device address of `scratch` per device, null until looked up

// The device address of the current device's copy of `scratch`, looked up
// once per device (with that device current) and kept.
int scratch_on_current_device(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return mmlttb::set_error(MMLTTB_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return mmlttb::set_error(MMLTTB_ENOTSUP, "device %d is beyond the %d devices the fixed scratch serves", dev,
                                 kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return mmlttb::set_error(MMLTTB_EDEVICE, "hipGetSymbolAddress of the fixed scratch failed on device %d: %s",
                                     dev, hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return MMLTTB_OK;
}

} // namespace

extern "C" {

int mmlttb_minmaxlttb_noalloc(int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps,
                              int64_t *out_idx, void *stream)
{
    const size_t need = mmlttb_workspace_size(n, n_out, r_ps);
    if (need == 0) // n_out or r_ps out of range: the checks of mmlttb_minmaxlttb name which
        return mmlttb_minmaxlttb(xk, x, y, n, n_out, r_ps, out_idx, nullptr, 0, stream);
    if (need > (size_t)MMLTTB_NOALLOC_SCRATCH_BYTES)
        return mmlttb::set_error(MMLTTB_EINVAL,
                                 "n_out=%lld with r_ps=%d needs %zu bytes of workspace; the fixed scratch of "
                                 "mmlttb_minmaxlttb_noalloc holds %zu (use mmlttb_minmaxlttb with a workspace)",
                                 (long long)n_out, (int)r_ps, need, (size_t)MMLTTB_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    const int rc = scratch_on_current_device(&ws);
    if (rc)
        return rc;
    return mmlttb_minmaxlttb(xk, x, y, n, n_out, r_ps, out_idx, ws, (size_t)MMLTTB_NOALLOC_SCRATCH_BYTES, stream);
}

} // extern "C"
