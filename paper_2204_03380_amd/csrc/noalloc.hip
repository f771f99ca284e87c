// The allocation-free variant of rtm_rtm_shot: its scratch is a fixed device
// array of this library instead of a caller workspace, for callers that
// cannot allocate device memory.  The array and every host use of its
// address live in this file.
#include <cstdint>
#include <cstdio>
#include <mutex>

#include <hip/hip_runtime.h>

#include "common.h"
#include "rtm.h"

// One array per GPU, held from the library's load until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it only stands for the symbol); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device with that device
// current.
static __device__ __align__(256) unsigned char scratch[RTM_NOALLOC_SCRATCH_BYTES];

namespace rtm {
int set_error(int code, const char *msg);  // the library's error state (api.hip)
void clear_error();
}  // namespace rtm

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int hip_fail(hipError_t e, const char *what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return rtm::set_error(RTM_EHIP, buf);
}

// Device address of the current device's scratch array.
int scratch_for_current_device(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return rtm::set_error(RTM_EHIP, "device index outside the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p & 255)) return rtm::set_error(RTM_EHIP, "scratch array not 256-byte aligned");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RTM_OK;
}

}  // namespace

extern "C" int rtm_rtm_shot_noalloc(const rtm_grid_t *grid, const float *v_pad, double dt, int32_t nt,
                                    const float *wavelet, const float *src, int32_t nrec, const float *rec,
                                    const float *traces, float eps_rel, float *image, float *num, float *den,
                                    uint32_t flags, void *stream)
{
    rtm::clear_error();
    size_t need = 0;
    int rc = rtm_workspace_bytes(grid, RTM_OP_RTM, nrec, nt, &need);
    if (rc) return rc;
    if (need > (size_t)RTM_NOALLOC_SCRATCH_BYTES) {
        char buf[256];
        snprintf(buf, sizeof buf,
                 "rtm_rtm_shot_noalloc: this shot needs %zu bytes of scratch, more than the library's fixed "
                 "%zu-byte array (use rtm_rtm_shot with a workspace)",
                 need, (size_t)RTM_NOALLOC_SCRATCH_BYTES);
        return rtm::set_error(RTM_EWORKSPACE, buf);
    }
    void *ws = nullptr;
    if ((rc = scratch_for_current_device(&ws))) return rc;
    return rtm_rtm_shot(grid, v_pad, dt, nt, wavelet, src, nrec, rec, traces, eps_rel, image, num, den, nullptr,
                        flags, ws, (size_t)RTM_NOALLOC_SCRATCH_BYTES, stream);
}
