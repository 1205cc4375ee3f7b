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

#include "prologue.h"
#include "sampler_launch.h"

namespace lens {

// The proposal and load kernels take a group of G = max(1, 256 / (7 nfree))
// consecutive walkers per block, whose parameters are contiguous: a thread
// per parameter of the group (proposal and prior test, coalesced), then a
// thread per potential (parameter prologue).  Each thread has one element of
// each phase (walkers with more than 36 free potentials loop), so every load
// round trip happens once per phase; the many small blocks fill the chip.
// The acceptance kernel takes one wave per walker, a lane per parameter.
constexpr int WALKERS_PER_BLOCK = 4;  // acceptance kernel

__host__ __device__ inline int walkers_per_group(int nfree) {
    return 7 * nfree >= 256 ? 1 : 256 / (7 * nfree);
}

// Physical parameters of one potential -> amplitude form -> derived
// constants at entry w*nfree + k: sigma [km/s] -> b0 [arcsec] = K pi
// (sigma/c)^2 rad, e -> eps = e/(1 + sqrt(1 - e^2)) (the same expressions as
// the table conversion), then the parameter prologue.
__device__ __forceinline__ void derive(const McmcArgs &a, int w, int k, const double q[7]) {
    const double c_kms = 299792.458;
    const double arcsec_per_rad = 648000.0 / M_PI;
    const double v = q[2] / c_kms;
    const double b0 = a.bK * M_PI * v * v * arcsec_per_rad;
    const double eps = q[3] / (1.0 + sqrt(1.0 - q[3] * q[3]));
    prologue_values(q[0], q[1], b0, eps, q[4], q[5], q[6], w * a.nfree + k, a.dd, a.df,
                    a.stride, a.status);
}

__global__ __launch_bounds__(256) void mcmc_load_kernel(McmcArgs a) {
    const int G = walkers_per_group(a.nfree);
    const int w0 = blockIdx.x * G, nw = min(G, a.W - w0);
    for (int e = threadIdx.x; e < nw * a.nfree; e += blockDim.x) {
        const int wl = e / a.nfree, k = e - wl * a.nfree, w = w0 + wl;
        const double *th = a.params + ((size_t)w * a.nfree + k) * 7;
        double q[7];
        for (int j = 0; j < 7; ++j) q[j] = th[j];
        derive(a, w, k, q);
    }
}

// Proposal and prior test per parameter; then the derived constants of each
// potential of the proposal (recomputed from the same inputs, so
// bit-identical to the stored proposal) or, when the walker's proposal is
// outside the box, of its current state, which keeps the table valid but is
// never used for a decision.
__global__ __launch_bounds__(256) void mcmc_propose_kernel(McmcArgs a) {
    __shared__ int outside[256];
    const int G = walkers_per_group(a.nfree);
    const int w0 = blockIdx.x * G, nw = min(G, a.W - w0);
    const int P = 7 * a.nfree;
    for (int t = threadIdx.x; t < nw; t += blockDim.x) outside[t] = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < nw * P; e += blockDim.x) {
        const int wl = e / P, i = e - wl * P, w = w0 + wl;
        const double v = a.params[(size_t)w * P + i] +
                         a.step[i] * (2.0 * a.u[(size_t)w * (P + 1) + i] - 1.0);
        a.prop[(size_t)w * P + i] = v;
        if (!(v >= a.lo[i] && v <= a.hi[i])) atomicOr(&outside[wl], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nw; t += blockDim.x) a.inside[w0 + t] = outside[t] ? 0 : 1;
    for (int e = threadIdx.x; e < nw * a.nfree; e += blockDim.x) {
        const int wl = e / a.nfree, k = e - wl * a.nfree, w = w0 + wl;
        const bool in = outside[wl] == 0;
        const double *th = a.params + (size_t)w * P + 7 * k;
        const double *uw = a.u + (size_t)w * (P + 1) + 7 * k;
        const double *sk = a.step + 7 * k;
        double q[7];
        for (int j = 0; j < 7; ++j) q[j] = in ? th[j] + sk[j] * (2.0 * uw[j] - 1.0) : th[j];
        derive(a, w, k, q);
    }
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
static dim3 groups_grid(int W, int nfree) {
    const int G = walkers_per_group(nfree);
    return dim3((unsigned)((W + G - 1) / G));
}

hipError_t launch_mcmc_load(const McmcArgs &a, hipStream_t st) {
    if (a.W <= 0) return hipSuccess;
    hipLaunchKernelGGL(mcmc_load_kernel, groups_grid(a.W, a.nfree), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_mcmc_propose(const McmcArgs &a, hipStream_t st) {
    if (a.W <= 0) return hipSuccess;
    hipLaunchKernelGGL(mcmc_propose_kernel, groups_grid(a.W, a.nfree), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_mcmc_accept(const McmcArgs &a, hipStream_t st) {
    if (a.W <= 0) return hipSuccess;
    hipLaunchKernelGGL(mcmc_accept_kernel, walkers_grid(a.W), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace lens
