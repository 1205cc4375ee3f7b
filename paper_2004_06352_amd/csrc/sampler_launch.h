// sampler_launch.h -- kernels of the Metropolis sampler (sampler.hip).
// Not part of the ABI.
#pragma once

#include "lens_internal.h"

namespace lens {

// Walkers' state and the step's buffers.  params/prop: [W][P] physical
// parameters (P = 7 nfree; per potential x0, y0, sigma, e, phi, rcore, rcut);
// amp: 7 planes of W*nfree amplitude-form entries (x0, y0, b0, eps, phi,
// rcore, rcut) evaluated by the chi^2 kernels.
struct McmcArgs {
    int W, nfree;
    double *params, *chi2;
    int *accepted;
    const double *lo, *hi, *step;  // [P]
    const double *u;               // [W][P + 1]
    double *prop;                  // [W][P]
    double *amp;                   // [7][W*nfree]
    int *inside;                   // [W]
    const double *chi2p;           // [W] chi^2 of the proposals
    double bK;                     // 6 (dPIE) or 4 (SIS)
};

// amp <- params (every walker's current state).
hipError_t launch_mcmc_load(const McmcArgs &a, hipStream_t st);
// prop <- params + step (2u - 1); inside <- prop within [lo, hi]; amp <- prop
// where inside, the current state elsewhere.
hipError_t launch_mcmc_propose(const McmcArgs &a, hipStream_t st);
// Metropolis decision per walker (chi2p from the chi^2 of amp).
hipError_t launch_mcmc_accept(const McmcArgs &a, hipStream_t st);

}  // namespace lens
