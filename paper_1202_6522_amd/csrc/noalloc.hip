// Synthesis without a caller workspace and without any allocation
// (shtn_synth_noalloc, include/shtn.h): the longitude coefficients F and the
// rescaled spectrum that shtn_synth keeps in its `work` argument live here in
// one static device array per GPU, loaded with the library's code object.
#include <hip/hip_runtime.h>

#include <mutex>

#include "shtn.h"
#include "shtn_internal.h"

namespace {

// Bytes of the static workspace: one field at lmax 1023 (24 MiB), five at
// lmax 511 or twenty at lmax 255 fit.
constexpr size_t kScratchBytes = SHTN_NOALLOC_MAX_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each GPU, looked up once per device with
// that device current.  The array's name is a host-side stand-in in host
// code: only these addresses may be passed to kernels.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

int scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return shtn::hip_error((int)e, "shtn_synth_noalloc: current device");
    if (dev < 0 || dev >= kMaxDevices) return shtn::set_error(SHTN_EUNSUPPORTED, "shtn_synth_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return shtn::hip_error((int)(e != hipSuccess ? e : hipErrorInvalidSymbol),
                                                           "shtn_synth_noalloc: static workspace address");
        g_addr[dev] = ptr;
    }
    *out = g_addr[dev];
    return SHTN_OK;
}

}  // namespace

extern "C" int shtn_synth_noalloc(shtn_plan_t plan, const double* Q, double* grid, int nfields, void* stream)
{
    if (!plan || !plan->p || nfields < 1) return shtn::set_error(SHTN_EINVAL, "null plan or nfields < 1");
    if (shtn_work_bytes(plan, nfields) > kScratchBytes)
        return shtn::set_error(SHTN_EINVAL, "shtn_synth_noalloc: the call needs more than the 32 MiB static "
                                            "workspace (use shtn_synth with a workspace)");
    void* ptr = nullptr;
    int rc = scratch_address(&ptr);
    if (rc) return rc;
    // Nothing in the workspace needs to start at zero: the kernels write
    // every entry of F and of the rescaled spectrum they later read, and the
    // padding behind the spectrum is loaded but never used.
    return shtn::synth_on_work(plan, Q, grid, nfields, ptr, stream);
}
