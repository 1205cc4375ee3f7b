// chi2.hip -- deflections at the constraint positions, the batched
// source-plane chi^2 (paper Sec. 2.2, Fig. 3 and Eq. (6): unlens every image
// with the lens equation of Sec. 2.1 Eq. (1), take each system's barycentre,
// sum the scatter over sigma^2) and the per-sample vertex deflection grids of
// the image-plane chi^2 (Sec. 4.2, stage 1).
//
// Design (gfx950): one 256-thread block per model sample.  Threads stride
// over the catalogue's images; the sample's free potentials are walked in
// index order with wave-uniform loads.  Unlensed positions go to LDS, then
// threads take one system each and the per-system sums are combined by
// shuffle reductions in a fixed order.  The batched path launches a few
// persistent blocks per CU that pull sample indices from a device counter
// until the batch is exhausted, so samples of uneven size balance across the
// chip; the per-sample path launches the same kernel once per sample.  Both
// produce bit-identical results.
#include <math.h>

#include "eval.h"

namespace lens {

// ---------------------------------------------------------------------------
// Fixed-potential deflection at the catalogue points, as partial sums over
// chunks of FIXED_CHUNK potentials: afix[(c*2 + {0,1})*nimg_pad + t].
// Summed by the consumer in chunk order (deterministic).

template <int PREC>
__global__ void __launch_bounds__(64) fixed_alpha_points_kernel(Derived tab, int nimg,
                                                                const double *__restrict__ X,
                                                                const double *__restrict__ Y,
                                                                int nimg_pad,
                                                                double *__restrict__ afix,
                                                                Series S) {
    const int t = blockIdx.x * 64 + threadIdx.x;
    const int c = blockIdx.y;
    const int k0 = c * FIXED_CHUNK, k1 = min(tab.n, k0 + FIXED_CHUNK);
    const double x = t < nimg ? X[t] : 0.0, y = t < nimg ? Y[t] : 0.0;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int k = k0; k < k1; ++k) {
        if (PREC == 0) {
            eval_pot_f64<true, false>(ConstD{tab.d + k, tab.stride}, x, y, acc, S);
        } else {
            float o[5];
            eval_pot_f32<true, false>(ConstD{tab.d + k, tab.stride},
                                      ConstF{tab.f + k, tab.stride}, x, y, o, S);
            acc[0] += (double)o[0];
            acc[1] += (double)o[1];
        }
    }
    if (t < nimg) {
        afix[((size_t)c * 2 + 0) * nimg_pad + t] = acc[0];
        afix[((size_t)c * 2 + 1) * nimg_pad + t] = acc[1];
    }
}

hipError_t launch_fixed_alpha_points(Derived fixedt, int nimg, const double *x, const double *y,
                                     int nchunk, int nimg_pad, double *afix, int prec,
                                     hipStream_t st) {
    if (nchunk <= 0 || nimg <= 0) return hipSuccess;
    dim3 grid((nimg + 63) / 64, nchunk);
    if (grid.y > 65535u) return hipErrorInvalidConfiguration;
    if (prec == 0)
        hipLaunchKernelGGL(fixed_alpha_points_kernel<0>, grid, dim3(64), 0, st, fixedt, nimg, x, y,
                           nimg_pad, afix, make_series());
    else
        hipLaunchKernelGGL(fixed_alpha_points_kernel<1>, grid, dim3(64), 0, st, fixedt, nimg, x, y,
                           nimg_pad, afix, make_series());
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ int system_of(const int *__restrict__ off, int nsys, int t) {
    int lo = 0, hi = nsys;  // off[lo] <= t < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// One block of SRC_BLOCK threads per sample: threads over images, then over
// systems; per-wave shuffle sums combined in a fixed order, so a sample's
// chi^2 does not depend on the batch it is evaluated in or on the path.
constexpr int SRC_BLOCK = 256;

template <int PREC>
__global__ void __launch_bounds__(SRC_BLOCK) chi2_src_kernel(Chi2SrcLaunch a) {
    extern __shared__ double sh[];  // [2][nimg]: unlensed x then y; then wave partials
    __shared__ int s_next;
    double *red = sh + 2 * (size_t)a.nimg;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int m = a.sample0 + blockIdx.x;
    for (;;) {
        if (a.persistent) {
            if (tid == 0) s_next = atomicAdd(a.queue, 1);
            __syncthreads();
            m = s_next;
        }
        if (m >= a.n_samples) break;
        const int nf = a.freet.n;
        const int k0 = min(max(a.free_off[m], 0), nf);
        const int k1 = min(max(a.free_off[m + 1], k0), nf);
        for (int t = tid; t < a.nimg; t += SRC_BLOCK) {
            const double x = a.x[t], y = a.y[t];
            double acc[5] = {0, 0, 0, 0, 0};
            for (int c = 0; c < a.nchunk; ++c) {
                acc[0] += a.afix[((size_t)c * 2 + 0) * a.nimg_pad + t];
                acc[1] += a.afix[((size_t)c * 2 + 1) * a.nimg_pad + t];
            }
            for (int k = k0; k < k1; ++k) {
                if (PREC == 0) {
                    eval_pot_f64<true, false>(ConstD{a.freet.d + k, a.freet.stride}, x, y, acc, a.S);
                } else {
                    float o[5];
                    eval_pot_f32<true, false>(ConstD{a.freet.d + k, a.freet.stride},
                                              ConstF{a.freet.f + k, a.freet.stride}, x, y, o, a.S);
                    acc[0] += (double)o[0];
                    acc[1] += (double)o[1];
                }
            }
            const double f = a.f[system_of(a.img_off, a.nsys, t)];
            sh[t] = x - f * acc[0];
            sh[a.nimg + t] = y - f * acc[1];
        }
        __syncthreads();
        double part = 0.0;
        for (int i = tid; i < a.nsys; i += SRC_BLOCK) {
            const int o0 = min(max(a.img_off[i], 0), a.nimg);
            const int o1 = min(max(a.img_off[i + 1], o0), a.nimg);
            const int M = o1 - o0;
            double mx = 0.0, my = 0.0;
            for (int t = o0; t < o1; ++t) {
                mx += sh[t];
                my += sh[a.nimg + t];
            }
            if (M > 0) {
                mx /= M;
                my /= M;
            }
            double s = 0.0;
            for (int t = o0; t < o1; ++t) {
                const double ex = sh[t] - mx, ey = sh[a.nimg + t] - my;
                s += (ex * ex + ey * ey) / (a.sig[t] * a.sig[t]);
            }
            part += s;
            if (a.src_x) {
                a.src_x[(size_t)m * a.nsys + i] = mx;
                a.src_y[(size_t)m * a.nsys + i] = my;
            }
        }
        part = wave_sum(part);
        if (lane == 0) red[wave] = part;
        __syncthreads();
        if (tid == 0 && a.chi2) {
            double total = red[0];
            for (int w = 1; w < SRC_BLOCK / 64; ++w) total += red[w];
            a.chi2[m] = total;
        }
        __syncthreads();
        if (!a.persistent) break;
    }
}

hipError_t launch_chi2_src(const Chi2SrcLaunch &c0, hipStream_t st) {
    Chi2SrcLaunch c = c0;
    c.S = make_series();
    const size_t shmem = ((size_t)2 * c.nimg + SRC_BLOCK / 64) * sizeof(double);
    if (c.prec == 0)
        hipLaunchKernelGGL(chi2_src_kernel<0>, dim3(c.grid_blocks), dim3(SRC_BLOCK), shmem, st, c);
    else
        hipLaunchKernelGGL(chi2_src_kernel<1>, dim3(c.grid_blocks), dim3(SRC_BLOCK), shmem, st, c);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Vertex deflection (Dls/Ds = 1) of samples m0 .. m0+nsamp-1: the fixed part
// (given) plus the sample's free potentials in index order.
template <int PREC>
__global__ void __launch_bounds__(256) alpha_grid_kernel(AlphaGridLaunch a) {
    const size_t nv = (size_t)a.grid.nx * a.grid.ny;
    const size_t v = (size_t)blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    const int m = a.m0 + s;
    const int nf = a.freet.n;
    const int k0 = min(max(a.free_off[m], 0), nf);
    const int k1 = min(max(a.free_off[m + 1], k0), nf);
    const int i = (int)(v % a.grid.nx), j = (int)(v / a.grid.nx);
    const double x = grid_coord(a.grid.x0, i, a.grid.dx);
    const double y = grid_coord(a.grid.y0, j, a.grid.dy);
    double acc[5] = {0, 0, 0, 0, 0};
    if (a.afix_x && v < nv) {
        acc[0] = a.afix_x[v];
        acc[1] = a.afix_y[v];
    }
    for (int k = k0; k < k1; ++k) {
        if (PREC == 0) {
            eval_pot_f64<true, false>(ConstD{a.freet.d + k, a.freet.stride}, x, y, acc, a.S);
        } else {
            float o[5];
            eval_pot_f32<true, false>(ConstD{a.freet.d + k, a.freet.stride},
                                      ConstF{a.freet.f + k, a.freet.stride}, x, y, o, a.S);
            acc[0] += (double)o[0];
            acc[1] += (double)o[1];
        }
    }
    if (v < nv) {
        a.out[(size_t)s * 2 * nv + v] = acc[0];
        a.out[(size_t)s * 2 * nv + nv + v] = acc[1];
    }
}

hipError_t launch_alpha_grid(const AlphaGridLaunch &L0, hipStream_t st) {
    AlphaGridLaunch L = L0;
    L.S = make_series();
    const size_t nv = (size_t)L.grid.nx * L.grid.ny;
    if (nv == 0 || L.nsamp <= 0) return hipSuccess;
    dim3 grid((unsigned)((nv + 255) / 256), L.nsamp);
    if (grid.y > 65535u) return hipErrorInvalidConfiguration;
    if (L.prec == 0)
        hipLaunchKernelGGL(alpha_grid_kernel<0>, grid, dim3(256), 0, st, L);
    else
        hipLaunchKernelGGL(alpha_grid_kernel<1>, grid, dim3(256), 0, st, L);
    return hipGetLastError();
}

}  // namespace lens
