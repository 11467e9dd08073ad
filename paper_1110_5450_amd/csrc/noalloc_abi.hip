// noalloc_abi.hip -- sweep_eval_noalloc: sweep_eval with its workspace in a
// static device array instead of caller memory, for callers that cannot
// allocate (code under graph capture, serving loops, harnesses that forbid
// hipMalloc).  The array belongs to the code object: every GPU the library
// runs on holds its own copy from module load to process exit.  Its device
// address is looked up once per device (hipGetSymbolAddress with that device
// current) and kept; host code never passes the array's own name to a kernel
// or a copy, since on the host that name is only a stand-in for the symbol.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/sweep.h"
#include "abi_internal.hpp"

namespace sweep {

static __device__ __align__(256) unsigned char scratch[SWEEP_NOALLOC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
static sweep_status scratch_of_current_device(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(SWEEP_ERR_UNSUPPORTED, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p) % 256 != 0) return fail(SWEEP_ERR_HIP, "scratch array address %p is not 256-byte aligned", p);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SWEEP_OK;
}

}  // namespace sweep

using namespace sweep;

extern "C" {

sweep_status sweep_eval_noalloc(const sweep_curve* path, const sweep_curve* profile, int32_t n_u, int32_t n_v,
                                const sweep_options* opt, void* pos, void* nrm, void* stream)
{
    sweep_options def;
    if (!opt) { sweep_default_options(&def); opt = &def; }
    // the same validation as sweep_eval, so that the size query below is
    // meaningful (it returns 0 for metadata sweep_eval would reject)
    sweep_status s = check_options(opt);
    if (s != SWEEP_OK) return s;
    if ((s = check_curve(path, "path", true)) != SWEEP_OK) return s;
    if ((s = check_curve(profile, "profile", false)) != SWEEP_OK) return s;
    if ((s = check_grid(n_u, n_v)) != SWEEP_OK) return s;
    const size_t need = sweep_eval_workspace_size(path, profile, n_u, n_v, opt);
    if (need > (size_t)SWEEP_NOALLOC_WORKSPACE_BYTES)
        return fail(SWEEP_ERR_WORKSPACE, "sweep_eval_noalloc: this sweep needs %zu bytes of workspace, the static array holds %zu",
                    need, (size_t)SWEEP_NOALLOC_WORKSPACE_BYTES);
    void* ws = nullptr;
    if ((s = scratch_of_current_device(&ws)) != SWEEP_OK) return s;
    return sweep_eval(path, profile, n_u, n_v, opt, pos, nrm, ws, (size_t)SWEEP_NOALLOC_WORKSPACE_BYTES, stream);
}

}  // extern "C"
