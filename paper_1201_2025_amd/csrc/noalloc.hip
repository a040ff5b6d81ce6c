// noalloc.hip -- hsad_detect for callers that cannot allocate device memory: the workspace
// comes from a static device array instead of the caller.
//
// Every GPU the library runs on holds its own copy of `scratch` (HSAD_NOALLOC_SCRATCH_BYTES)
// from the loading of the code object until the process ends.  In host code the array's
// name is only a host-side handle, so the device address of each GPU's copy is looked up
// once per device (hipGetSymbolAddress, with that device current) and only that address is
// ever handed to kernels.  hsad_detect's kernels write every workspace byte they read
// before reading it, so nothing has to be cleared between calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace hsad {

static __device__ __align__(256) unsigned char scratch[HSAD_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_ptr;   // device ordinal -> address of its copy

// Device address of the current device's copy of `scratch` (nullptr and an error message
// when the lookup fails).
static void *scratch_address(int *rc)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        *rc = fail(HSAD_EHIP, "hsad_detect_noalloc: hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) return it->second;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        *rc = fail(HSAD_EHIP, std::string("hsad_detect_noalloc: hipGetSymbolAddress(scratch): ") +
                                  hipGetErrorString(e));
        return nullptr;
    }
    g_scratch_ptr.emplace(dev, ptr);
    return ptr;
}

}  // namespace hsad

using namespace hsad;

extern "C" int hsad_detect_noalloc(const float *x, int64_t H, int64_t W, int64_t Lp,
                                   const hsad_window_params *p, double z_alpha, float *lrx,
                                   float *dwrx, double *stats, uint8_t *mask, hipStream_t stream)
{
    clear_error();
    const size_t need = detect_min_bytes(H, W, Lp, p, dwrx != nullptr);
    if (need == 0)   // invalid arguments: hsad_detect reports them without launching anything
        return hsad_detect(x, H, W, Lp, p, z_alpha, lrx, dwrx, stats, mask, nullptr, 0, stream);
    if (!x || !lrx || !stats) return fail(HSAD_EINVAL, "hsad_detect_noalloc: x, lrx and stats are required");
    if (!std::isfinite(z_alpha)) return fail(HSAD_EINVAL, "hsad_detect_noalloc: z_alpha not finite");
    if (need > (size_t)HSAD_NOALLOC_SCRATCH_BYTES)
        return fail(HSAD_ENOMEM, "hsad_detect_noalloc: this image needs " + std::to_string(need) +
                                     " bytes of workspace, more than the static scratch of " +
                                     std::to_string((size_t)HSAD_NOALLOC_SCRATCH_BYTES) + " bytes");
    int rc = HSAD_OK;
    void *ws = scratch_address(&rc);
    if (!ws) return rc;
    size_t want = hsad_detect_workspace_bytes(H, W, Lp, p);
    if (want > (size_t)HSAD_NOALLOC_SCRATCH_BYTES) want = HSAD_NOALLOC_SCRATCH_BYTES;
    if (want < need) want = need;
    return hsad_detect(x, H, W, Lp, p, z_alpha, lrx, dwrx, stats, mask, ws, want, stream);
}
