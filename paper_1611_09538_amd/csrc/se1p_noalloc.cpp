// se1p_noalloc.cpp -- se1p_eval_noalloc: the evaluation of se1p_eval with its
// per-call scratch in a static device array instead of the plan's workspace,
// for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "se1p_plan.h"

using namespace se1p;

// The scratch: a file-scope device array, one copy on every GPU the library
// runs on, held until the process ends.  In host code the array's name is
// not a device address: its address on each device is looked up once, with
// that device current, by hipGetSymbolAddress and kept per device, and only
// that address is used (as the base of the buffers handed to the kernels).
static __device__ __align__(256) unsigned char scratch[SE1P_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the static scratch on device dev (made current by the
// caller): looked up on the first call on that device.
int static_scratch(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return SE1P_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SE1P_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SE1P_OK;
}

// Points the plan's scratch at another layout for the duration of a call
// and restores the plan's own when the call returns.
struct ScratchSwap {
    se1p_plan& pl;
    PlanScratch saved;
    ScratchSwap(se1p_plan& p, const PlanScratch& w) : pl(p), saved(p.w) { pl.w = w; }
    ~ScratchSwap() { pl.w = saved; }
};

}  // namespace

extern "C" int se1p_eval_noalloc(se1p_plan* pl, long long N, const void* x,
                                 const void* q, void* phi, void* efield,
                                 double* energy, unsigned flags) {
    int rc = eval_args(pl, N, x, q, flags);
    if (rc) return rc;
    // the layout of this call (sizes from the plan's geometry and N only)
    PlanScratch w;
    const bool ik = (flags & SE1P_FIELD_IK) != 0;
    if (layout_scratch(*pl, N, w, 0, ik) > (size_t)SE1P_NOALLOC_SCRATCH_BYTES)
        return SE1P_ERR_SCRATCH;
    if (set_device(pl)) return SE1P_ERR_HIP;
    void* base = nullptr;
    if ((rc = static_scratch(pl->device, &base))) return rc;
    layout_scratch(*pl, N, w, (uintptr_t)base, ik);
    ScratchSwap swap(*pl, w);
    return eval_body(pl, N, x, q, phi, efield, energy, flags);
}
