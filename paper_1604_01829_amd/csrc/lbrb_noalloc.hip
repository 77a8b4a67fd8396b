// lbrb_noalloc.hip -- the reverse pass on a scratch array of the library, for callers that
// cannot allocate device memory.
//
// lb_rb_adjoint runs on a workspace the caller passes.  lb_rb_adjoint_noalloc runs the same
// code on `scratch`, a file-scope device array of LB_NOALLOC_SCRATCH_BYTES that every GPU the
// library runs on holds until the process ends.  In host code the array's name is only a
// stand-in for the symbol: its device address is taken once per device with
// hipGetSymbolAddress (at lb_init, with that device current, or at the first call on a
// device) and only that address is ever passed on.  Every call on one GPU uses that GPU's
// array; lb_rb_adjoint clears the parts that must start at zero, so the previous call's
// contents do not matter, but calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lbrb.h"

namespace lbrb {
int set_error(lb_ctx* c, int code, const char* msg);   // lbrb_api.cpp
}

namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[LB_NOALLOC_SCRATCH_BYTES];

std::mutex g_lock;
void* g_scratch[kMaxDevices] = {};

// the device address of this device's array (nullptr if HIP refuses it)
void* scratch_address(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_lock);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

}  // namespace

namespace lbrb {

// take the address on the current device (called by lb_init)
void noalloc_prepare()
{
    int dev = -1;
    if (hipGetDevice(&dev) == hipSuccess) (void)scratch_address(dev);
}

}  // namespace lbrb

extern "C" int lb_rb_adjoint_noalloc(lb_ctx* ctx, int32_t n_steps, int32_t checkpoint_every,
                                     const double* dJ_dF, double* J, double* dJ_dgamma,
                                     double* dJ_doffsets)
{
    if (!ctx) return LB_ERR_ARG;
    const size_t need = lb_adjoint_workspace_bytes(ctx, n_steps, checkpoint_every);
    if (need == 0)
        return lbrb::set_error(ctx, LB_ERR_ARG,
                               "the window needs n_steps >= 1 and checkpoint_every >= 1");
    if (need > (size_t)LB_NOALLOC_SCRATCH_BYTES)
        return lbrb::set_error(ctx, LB_ERR_ARG,
                               "the reverse pass needs more than LB_NOALLOC_SCRATCH_BYTES: use "
                               "lb_rb_adjoint with a workspace, or a longer checkpoint interval");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return lbrb::set_error(ctx, LB_ERR_HIP, "hipGetDevice");
    void* ws = scratch_address(dev);
    if (!ws) return lbrb::set_error(ctx, LB_ERR_HIP, "hipGetSymbolAddress of the scratch array");
    return lb_rb_adjoint(ctx, n_steps, checkpoint_every, ws, (size_t)LB_NOALLOC_SCRATCH_BYTES,
                         dJ_dF, J, dJ_dgamma, dJ_doffsets);
}
