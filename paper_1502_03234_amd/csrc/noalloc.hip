// noalloc.hip -- the smoothing stage (periodic [1,2,1] passes per axis) for callers that cannot
// allocate device memory: code under graph capture, tight serving loops, hosts that forbid it.
//
// The passes ping-pong between the output image and one intermediate image. dcm_grid_smooth
// takes that intermediate from the caller's workspace; dcm_grid_smooth_noalloc takes it from
// `scratch`, a file-scope device array of kNoallocBoxes entries (32 MiB) that every device the
// library runs on holds until the process ends. Host code never passes the array's name to a
// kernel (in host code it names a host-side stand-in): the device address is looked up once per
// device with hipGetSymbolAddress, with that device current, and kept.
//
// Every call on one device shares that device's array: calls that overlap on one device (two
// streams, two threads) race and corrupt each other's intermediate image. Each smoothing pass
// writes every box of its output, so nothing needs clearing between calls.
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "internal.h"

namespace dcm {
namespace {

constexpr int64_t kNoallocBoxes = (int64_t)1 << 23;   // 8,388,608 boxes
static __device__ __align__(256) uint32_t scratch[kNoallocBoxes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];                      // per device; nullptr until looked up

// Device address of the current device's scratch array.
dcm_status scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report_error(DCM_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return report_error(DCM_E_HIP, "device %d outside 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return report_error(DCM_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DCM_OK;
}

}  // namespace
}  // namespace dcm

using namespace dcm;

extern "C" dcm_status dcm_grid_smooth_noalloc(const int32_t dims[3], int32_t passes, const uint32_t *d_in,
                                              uint32_t *d_out, dcm_stream_t stream)
{
    if (!dims) return report_error(DCM_E_INVALID, "dims is NULL");
    Grid g = {};
    for (int k = 0; k < 3; ++k) {
        if (dims[k] < 3) return report_error(DCM_E_INVALID, "every grid dimension must be >= 3");
        g.n[k] = dims[k];
        g.h[k] = 1.0;
        g.L[k] = dims[k];
    }
    g.G = (int64_t)dims[0] * dims[1] * dims[2];
    if (g.G > kNoallocBoxes)
        return report_error(DCM_E_INVALID, "grid of %lld boxes exceeds the %lld boxes of the no-allocation scratch",
                            (long long)g.G, (long long)kNoallocBoxes);
    if (passes < 0 || passes > 4) return report_error(DCM_E_INVALID, "passes must be 0..4");
    if (!d_in || !d_out) return report_error(DCM_E_INVALID, "NULL image");
    void *tmp = nullptr;
    dcm_status rs = scratch_address(&tmp);
    if (rs != DCM_OK) return rs;
    launch_smooth(g, passes, nullptr, d_in, d_out, (uint32_t *)tmp, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return report_error(DCM_E_HIP, "dcm_grid_smooth_noalloc: %s", hipGetErrorString(e));
    return DCM_OK;
}
