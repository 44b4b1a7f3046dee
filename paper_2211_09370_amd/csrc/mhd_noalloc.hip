// Allocation-free stepping for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc): mhd_step_noalloc runs the same
// kernels as mhd_step with their scratch (Lorentz force, wall corrections, flow and budget
// partials) in one file-scope device array of this library instead of the solver's workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mhd_internal.h"

using namespace mhd;

namespace {

// Maximum step scratch: 32 MiB, enough for boxes up to about 2.7 M cells (the 128^3 box needs
// 25.3 MB). Each GPU the library runs on holds its own copy until the process ends.
constexpr size_t kScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per device with that device
// current (the array's name in host code is only a host-side stand-in for the symbol).
mhd_status scratch_for(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return report_error(MHD_ERR_UNSUPPORTED, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return report_error(MHD_ERR_HIP, "hipGetSymbolAddress of the step scratch failed");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MHD_OK;
}

}  // namespace

extern "C" mhd_status mhd_step_noalloc(mhd_sim *s, int64_t n_steps, int32_t budget_every) {
    (void)report_error(MHD_OK, "");
    mhd_status st = step_checks(s, n_steps);
    if (st != MHD_OK) return st;
    if (step_scratch_bytes(s) > kScratchBytes)
        return report_error(MHD_ERR_INVALID_ARG,
                            "box too large for mhd_step_noalloc: its step scratch exceeds the 32 MiB static buffer "
                            "(about 2.7 M cells); use mhd_step");
    void *p = nullptr;
    st = scratch_for(sim_device(s), &p);
    if (st != MHD_OK) return st;
    return step_in_scratch(s, n_steps, budget_every, p);
}
