// xy_noalloc.hip -- xy_label_links_noalloc: the standalone labelling of a
// given link set (the same kernels as xy_label_links) with its scratch in a
// fixed device array of this library instead of memory allocated per call,
// for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "../../include/xy.h"
#include "xy_device.hpp"
#include "xy_host.hpp"
#include "xy_launch.hpp"

namespace {

// Scratch of every call on a device: state and descriptor, tile-local labels,
// edge slots, the forest of boundary components and the edge-link masks
// (14 MiB at L = 2048 with 16-row tiles, the largest case).
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device, taken once per device with that
// device current.  In host code the array's name is only a host-side stand-in.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_scratch[kMaxDevices] = {};

int scratch_of_current_device(char **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return xyhost::fail(XY_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    }
    if (dev < 0 || dev >= kMaxDevices) return xyhost::fail(XY_EDEVICE, "device %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return xyhost::fail(XY_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                                hipGetErrorString(e));
        }
        g_scratch[dev] = static_cast<char *>(p);
    }
    *out = g_scratch[dev];
    return XY_OK;
}

// Writes the descriptor (passed by value, no host copy) and a zeroed replica
// state into the scratch.
__global__ void k_setup_labelling(xy::RepDesc d, xy::RepDesc *desc_out, xy::RepState *st_out)
{
    constexpr int nst = (int)(sizeof(xy::RepState) / sizeof(uint32_t));
    static_assert(sizeof(xy::RepState) % sizeof(uint32_t) == 0, "state size");
    uint32_t *w = reinterpret_cast<uint32_t *>(st_out);
    for (int k = threadIdx.x; k < nst; k += blockDim.x) w[k] = 0u;
    if (threadIdx.x == 0) *desc_out = d;
}

}  // namespace

extern "C" int xy_label_links_noalloc(int64_t L, int32_t label_bits, int32_t tile_rows, const uint32_t *d_bx,
                                      const uint32_t *d_by, void *d_labels, void *hip_stream)
{
    if (!d_bx || !d_by || !d_labels) return xyhost::fail(XY_EINVAL, "device pointer is NULL");
    xyhost::LinkLabelJob J;
    int rc = xyhost::plan_link_labels(L, label_bits, tile_rows, J);
    if (rc) return rc;
    if (J.total > kScratchBytes)
        return xyhost::fail(XY_EINVAL,
                            "L=%lld with %d-row tiles needs %zu bytes of scratch, more than the %zu bytes of the "
                            "library's fixed scratch (L <= 2048 fits)",
                            (long long)L, J.plan.res[0].TH, J.total, kScratchBytes);
    char *mem = nullptr;
    rc = scratch_of_current_device(&mem);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    xy::RepDesc d;
    xyhost::link_label_desc(J, mem, d_bx, d_by, d);
    hipLaunchKernelGGL(k_setup_labelling, dim3(1), dim3(64), 0, s, d,
                       reinterpret_cast<xy::RepDesc *>(mem + J.off_desc),
                       reinterpret_cast<xy::RepState *>(mem + J.off_state));
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = xyhost::enqueue_link_labels(J, mem, d_labels, s);
    if (e != hipSuccess) return xyhost::fail(XY_EDEVICE, "labelling failed: %s", hipGetErrorString(e));
    return XY_OK;
}
