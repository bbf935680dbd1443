// kgs_step_fields: DP-AVF2 steps on caller-owned fields without any device
// allocation.  The colour-split state (and, where it fits, the second buffer
// of the ping-pong kernels) lives in one fixed scratch array per device.
//
// The array's name is a host-side stand-in in host code; its device address
// comes from hipGetSymbolAddress, looked up once per device with that device
// current and kept per device.  Only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "kgs.h"
#include "kgs_trace.h"
#include "kgs_sim.h"

namespace {

static __device__ __align__(256) unsigned char scratch[KGS_STEP_FIELDS_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch`, per device id

// Device address of the scratch array on the current device.
int scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return kgs::set_error(KGS_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorName(e));
    if (dev < 0 || dev >= kMaxDevices)
        return kgs::set_error(KGS_EDEVICE, "device id " + std::to_string(dev) +
                                               " beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return kgs::set_error(KGS_EDEVICE, std::string("hipGetSymbolAddress (scratch): ") +
                                                   hipGetErrorName(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return KGS_OK;
}

}  // namespace

extern "C" int kgs_step_fields(const kgs_config *cfg, double *psi_re, double *psi_im, double *u,
                               double *v_t, int64_t nsteps, void *stream)
{
    KGS_TRACE("kgs_step_fields");
    int rc = kgs::step_fields_check(cfg, psi_re, psi_im, u, v_t, nsteps,
                                    KGS_STEP_FIELDS_SCRATCH_BYTES);
    if (rc != KGS_OK) return rc;
    void *p = nullptr;
    rc = scratch_address(&p);
    if (rc != KGS_OK) return rc;
    return kgs::step_fields_run(cfg, psi_re, psi_im, u, v_t, nsteps,
                                static_cast<hipStream_t>(stream), p,
                                KGS_STEP_FIELDS_SCRATCH_BYTES);
}
