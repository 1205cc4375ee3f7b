// sampler_launch.h -- kernels of the Metropolis sampler (sampler.hip).
// Not part of the ABI.
#pragma once

#include "lens_internal.h"

namespace lens {

// Walkers' state and the step's buffers.  params/prop: [W][P] physical
// parameters (P = 7 nfree; per potential x0, y0, sigma, e, phi, rcore, rcut).
// The derived table (W*nfree entries, walker w's potentials at w*nfree ..)
// is what the chi^2 kernels evaluate.
struct McmcArgs {
    int W, nfree;
    double *params, *chi2;
    int *accepted;
    const double *lo, *hi, *step;  // [P]
    const double *u;               // [W][P + 1]
    double *prop;                  // [W][P]
    int *inside;                   // [W]
    const double *chi2p;           // [W] chi^2 of the proposals
    double *dd;                    // derived table, FP64 block
    float *df;                     // derived table, FP32 block
    int stride;                    // its stride (>= W*nfree)
    int *status;                   // status word (invalid parameters)
    double bK;                     // 6 (dPIE) or 4 (SIS)
};

// derived table <- params (every walker's current state).
hipError_t launch_mcmc_load(const McmcArgs &a, hipStream_t st);
// prop <- params + step (2u - 1); inside <- prop within [lo, hi]; derived
// table <- prop where inside, the current state elsewhere.
hipError_t launch_mcmc_propose(const McmcArgs &a, hipStream_t st);
// Metropolis decision per walker (chi2p from the chi^2 of the derived table).
hipError_t launch_mcmc_accept(const McmcArgs &a, hipStream_t st);

}  // namespace lens
