// potential_launch.h -- launch wrapper of the potential / time-delay map
// kernel (potential.hip).  Not part of the ABI.
#pragma once

#include "lens_internal.h"

namespace lens {

// td = 0: out = dlsds * psi; td = 1: out = scale (|theta - beta|^2 / 2 - dlsds * psi).
hipError_t launch_potential_map(Derived tab, GridArgs g, double dlsds, double *out, int td,
                                double bx, double by, double scale, hipStream_t st);

}  // namespace lens
