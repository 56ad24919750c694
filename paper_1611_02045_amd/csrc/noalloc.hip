// H_phi apply that allocates nothing: the transform intermediate of the two directional passes
// lives in a file-scope device array instead of the plan's growable workspace.
#include <cstring>
#include <mutex>
#include <string>

#include "internal.hpp"
#include "plan.hpp"

namespace {

// Largest intermediate of one call: count * N complex values of the plan's precision.
constexpr size_t kScratchBytes = GPE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Each device holds its own copy of the array for the life of the process.  Host code never
// names it in a launch or copy: it uses the device address obtained once per device below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first call per device.
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

using namespace gpe;

extern "C" {

int gpe_apply_H_batched_noalloc(gpe_plan_t* plan, int count, const void* phi, const void* V, void* Hphi,
                                void* stream) {
    if (!plan || !phi || !V || !Hphi) {
        set_error("plan, phi, V and Hphi must not be NULL");
        return GPE_EINVAL;
    }
    if (count < 1) { set_error("count must be >= 1"); return GPE_EINVAL; }
    if (phi == Hphi) { set_error("Hphi must not alias phi"); return GPE_EINVAL; }
    const size_t cb = plan->f64() ? 16 : 8;
    const size_t need = cb * (size_t)plan->g.N * (size_t)count;
    if (need > kScratchBytes) {
        set_error("count * N complex values exceed the static scratch of " + std::to_string(kScratchBytes >> 20) +
                  " MiB (" + std::to_string(need) + " bytes needed)");
        return GPE_EINVAL;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && dev != plan->device) {
        set_error("the plan belongs to another device than the current one");
        return GPE_EINVAL;
    }
    void* tmp = nullptr;
    if (e == hipSuccess) e = scratch_address(&tmp);
    if (e == hipSuccess)
        e = op_apply(plan->g, plan->f64(), count, plan->tw, phi, V, Hphi, tmp, plan->prob.beta, plan->prob.omega,
                     true, (hipStream_t)stream);
    if (e != hipSuccess) {
        set_error(std::string("HIP error in gpe_apply_H_batched_noalloc: ") + hipGetErrorString(e));
        return GPE_EHIP;
    }
    return GPE_OK;
}

}  // extern "C"
