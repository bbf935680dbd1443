// Host-side state of a simulation handle (shared by the single-simulation
// API, the batch API and the server; not part of the public ABI).
#pragma once

#include <cstdint>
#include <string>

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
    double *host_out = nullptr;  // pinned, 2 doubles
    hipStream_t stream = nullptr;
    int device = 0;
    kgs_tuning tuning;
    int64_t device_bytes = 0;
    std::string err;
};
