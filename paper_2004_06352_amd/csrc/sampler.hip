// sampler.hip -- proposal and acceptance kernels of the Metropolis sampler
// around the batched source-plane chi^2 (Sec. 2.2: the parameter space is
// explored by a Bayesian MCMC; Sec. 4 names the sampler the third
// bottleneck).  The chi^2 of all proposals is one batched evaluation between
// the two kernels.
//
// Compiled with -ffp-contract=off: a proposal theta + step (2u - 1) and the
// parameter conversions are the same rounded operations as anywhere else
// they are written, so walkers given the same uniforms propose bit-identical
// parameters.
#include <math.h>

#include "sampler_launch.h"

namespace lens {

// One wave per walker, a lane per parameter (strided by 64 when a walker has
// more than nine free potentials): the walker's parameters, uniforms, box and
// proposal are read and written coalesced.
constexpr int WALKERS_PER_BLOCK = 4;

// Amplitude-form value of physical parameter j of a potential: sigma [km/s]
// -> b0 [arcsec] = K pi (sigma/c)^2 rad, e -> eps = e/(1 + sqrt(1 - e^2)),
// the others as they are (the same expressions as the parameter prologue's
// conversion).
__device__ __forceinline__ double to_amp(double q, int j, double bK) {
    const double c_kms = 299792.458;
    const double arcsec_per_rad = 648000.0 / M_PI;
    if (j == 2) {
        const double v = q / c_kms;
        return bK * M_PI * v * v * arcsec_per_rad;
    }
    if (j == 3) return q / (1.0 + sqrt(1.0 - q * q));
    return q;
}

__device__ __forceinline__ void store_amp(const McmcArgs &a, int w, int i, double q) {
    const int k = i / 7, j = i - 7 * k;
    const size_t n = (size_t)a.W * a.nfree;
    a.amp[j * n + (size_t)w * a.nfree + k] = to_amp(q, j, a.bK);
}

__global__ __launch_bounds__(256) void mcmc_load_kernel(McmcArgs a) {
    const int w = blockIdx.x * WALKERS_PER_BLOCK + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= a.W) return;
    const int P = 7 * a.nfree;
    for (int i = lane; i < P; i += 64) store_amp(a, w, i, a.params[(size_t)w * P + i]);
}

__global__ __launch_bounds__(256) void mcmc_propose_kernel(McmcArgs a) {
    const int w = blockIdx.x * WALKERS_PER_BLOCK + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= a.W) return;
    const int P = 7 * a.nfree;
    const double *th = a.params + (size_t)w * P;
    const double *uw = a.u + (size_t)w * (P + 1);
    double *pr = a.prop + (size_t)w * P;
    int out = 0;
    for (int i = lane; i < P; i += 64) {
        const double v = th[i] + a.step[i] * (2.0 * uw[i] - 1.0);
        pr[i] = v;
        if (!(v >= a.lo[i] && v <= a.hi[i])) out = 1;
    }
    const bool in = __ballot(out) == 0;
    if (lane == 0) a.inside[w] = in ? 1 : 0;
    // an out-of-prior proposal is never evaluated: its slot holds the current
    // (valid) state
    const double *src = in ? pr : th;
    for (int i = lane; i < P; i += 64) store_amp(a, w, i, src[i]);
}

// Accept when chi2' <= chi2 or -2 ln u_last > chi2' - chi2: probability
// min(1, exp(-(chi2' - chi2)/2)) for the likelihood exp(-chi2/2).
__global__ __launch_bounds__(256) void mcmc_accept_kernel(McmcArgs a) {
    const int w = blockIdx.x * WALKERS_PER_BLOCK + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= a.W) return;
    const int P = 7 * a.nfree;
    const double c = a.chi2[w], cp = a.chi2p[w];
    const double d = cp - c;
    const double ul = a.u[(size_t)w * (P + 1) + P];
    if (a.inside[w] && (d <= 0.0 || -2.0 * log(ul) > d)) {
        for (int i = lane; i < P; i += 64)
            a.params[(size_t)w * P + i] = a.prop[(size_t)w * P + i];
        if (lane == 0) {
            a.chi2[w] = cp;
            a.accepted[w] += 1;
        }
    }
}

static dim3 walkers_grid(int W) {
    return dim3((unsigned)((W + WALKERS_PER_BLOCK - 1) / WALKERS_PER_BLOCK));
}

hipError_t launch_mcmc_load(const McmcArgs &a, hipStream_t st) {
    if (a.W <= 0) return hipSuccess;
    hipLaunchKernelGGL(mcmc_load_kernel, walkers_grid(a.W), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_mcmc_propose(const McmcArgs &a, hipStream_t st) {
    if (a.W <= 0) return hipSuccess;
    hipLaunchKernelGGL(mcmc_propose_kernel, walkers_grid(a.W), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_mcmc_accept(const McmcArgs &a, hipStream_t st) {
    if (a.W <= 0) return hipSuccess;
    hipLaunchKernelGGL(mcmc_accept_kernel, walkers_grid(a.W), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace lens
