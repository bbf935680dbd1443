// The energy reduction that first applies the sweep closing a step
// (kgs_energy.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include "kgs_internal.h"

namespace kgs {

// The adjoint red sweep (PASS_R_ADJ with constants kc, in place) and then
// E_h of the swept state into out[0..1], in one pass over the state: the
// state ends bitwise as after launch_sweep(PASS_R_ADJ) and out holds
// bitwise what launch_energy gives on that state.  hipErrorNotSupported for
// grids that launch_energy does not stream (1-D, or 3-D beyond 1024 points
// per axis): sweep, then launch_energy, instead.
hipError_t launch_energy_closing(const Geometry &g, int precision, void *state,
                                 const EnergyCoef &k, const Coef &kc, double *partials,
                                 double *out, hipStream_t s);

}  // namespace kgs
