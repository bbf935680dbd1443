// Host-side state of a simulation handle (shared by the single-simulation
// API, the batch API and the server; not part of the public ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "kgs.h"
#include "kgs_internal.h"

struct kgs_sim {
    kgs_config cfg;
    kgs::Geometry geo;
    double h;
    double hd;             // h^dim
    kgs::Coef coef;        // constants of one half step (tau/2)
    kgs::EnergyCoef ecoef;
    void *state = nullptr; // 8 colour-split planes
    void *state2 = nullptr; // second copy for ping-pong kernels (3-D streaming)
    size_t plane_bytes = 0;
    double *partials = nullptr;  // energy partials, then the 2-double result
    double *host_out = nullptr;  // pinned, 2 doubles (not held by pooled handles)
    hipMemPool_t pool = nullptr; // device memory comes from this pool in stream order
    hipStream_t stream = nullptr;
    int device = 0;
    kgs_tuning tuning;
    int64_t device_bytes = 0;
    // the adjoint red sweep that closes the last step is still to be
    // applied (kgs_step leaves it to the next step, which fuses it with its
    // first red sweep, or to the next call that reads the state)
    bool open = false;
    std::string err;
};

namespace kgs {

// Applies a handle's pending adjoint red sweep (if any) on `stream`.
int sim_close(kgs_sim *s, hipStream_t stream);

// The first failure of a series of runtime calls that are all attempted,
// such as the releases of every resource of an object, which continue after
// one of them has failed.
struct FirstError {
    hipError_t e = hipSuccess;
    void operator()(hipError_t x)
    {
        if (e == hipSuccess) e = x;
    }
    bool ok() const { return e == hipSuccess; }
};

// Handles for the server: device memory from `pool` in the order of `stream`
// (no host synchronisation anywhere), initial state from float64 device
// arrays read by a scatter kernel on the stream, the library's default
// launch configuration.  kgs_step / kgs_set_tuning work on such handles;
// kgs_energy does not (the caller launches the energy kernel itself).
int sim_create_pooled(const kgs_config *cfg, const double *P, const double *Q, const double *U,
                      const double *V, hipStream_t stream, hipMemPool_t pool, kgs_sim **out,
                      std::string &err);
// Returns the memory to the pool in stream order after all queued work.
void sim_destroy_pooled(kgs_sim *s);
// KGS_KERNEL_* that a new handle for cfg (valid) runs by default.
int default_kernel(const kgs_config &cfg);
// The library's launch configuration for cfg (what KGS_KERNEL_AUTO picks).
kgs_tuning default_tuning_of(const kgs_config &cfg);
// Give the handle its second state buffer (ping-pong kernels) if it has none.
int sim_ensure_state2(kgs_sim *s);
// Launch configuration of a streaming group in a batch: mode GROUP_STREAM2D
// (y-streaming, rows per task `chunk`), GROUP_TILE2D (tiles of ty rows x
// tx compressed positions) or GROUP_STREAM3D (z-streaming over a member
// list, planes per workgroup `chunk`).
enum { GROUP_STREAM2D = 0, GROUP_TILE2D = 1, GROUP_STREAM3D = 2 };
struct GroupTuning {
    int mode = GROUP_STREAM2D, chunk = 0, ty = 0, tx = 0;
};
// Tuned group configurations (kgs_tune.cpp): the signature of a group
// (architecture of the device, dimension, precision, sorted member sizes),
// and a cache of winners in this process and, when KGS_TUNE_CACHE names a
// file, in that file.
std::string group_signature(int device, int dim, int precision, std::vector<int> sizes);
bool group_cache_get(const std::string &sig, GroupTuning &t);
void group_cache_put(const std::string &sig, const GroupTuning &t);
// Bytes of one state buffer (8 planes) of a valid cfg.
int64_t state_bytes(const kgs_config &cfg);
// Sets the calling thread's last error (kgs_last_error(NULL)); returns code.
int set_error(int code, const std::string &msg);
// kgs_step_fields, host side: argument and size checks (nothing touches
// the device), then scatter, kgs_step's launches and gather on `stream`
// with the state in `scratch` (device memory of scratch_bytes).
int step_fields_check(const kgs_config *cfg, const double *P, const double *Q, const double *U,
                      const double *V, int64_t nsteps, int64_t scratch_bytes);
int step_fields_run(const kgs_config *cfg, double *P, double *Q, double *U, double *V,
                    int64_t nsteps, hipStream_t stream, void *scratch, int64_t scratch_bytes);

}  // namespace kgs
