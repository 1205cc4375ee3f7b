// maps.hip -- parameter prologue and the fused deflection / second-derivative
// map kernel (paper Sec. 4.1 Eq. (10): the map is, at every grid point, the
// sum over potentials of each potential's derivatives; Sec. 2.4 Eqs. (7)-(9)
// for the second derivatives).
//
// Design (gfx950): one thread per grid point (or pix_per_thread points along
// x, strided by block_x so that each wave stores 64 consecutive pixels);
// every lane of the block walks the potentials in index order, so each
// potential's constants are uniform across the wave.  They are either staged
// through LDS in chunks (stage = 1, broadcast reads) or read with wave-uniform
// loads (stage = 0).  Accumulators stay in registers; each output channel is a
// row-major plane written once with coalesced stores.
#include <math.h>

#include "eval.h"
#include "prologue.h"

namespace lens {

// ---------------------------------------------------------------------------
__global__ void zero_i32_kernel(int *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_zero_i32(int *p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

__global__ void fill_f64_kernel(double *p, size_t n, double v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void fill_i64_kernel(long long *p, size_t n, long long v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
hipError_t launch_fill_f64(double *p, size_t n, double v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p,
                       n, v);
    return hipGetLastError();
}
hipError_t launch_fill_i64(long long *p, size_t n, long long v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p,
                       n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Physical -> amplitude form.  b0 = K pi (sigma/c)^2 rad in arcsec, K = 6
// (Lenstool dPIE) or 4 (singular isothermal sphere); eps from e as
// e / (1 + sqrt(1 - e^2)), the cancellation-free form of (1 - sqrt(1-e^2))/e.
__global__ void phys_to_amp_kernel(const double *__restrict__ sigma, const double *__restrict__ e,
                                   int n, double K, double *__restrict__ b0,
                                   double *__restrict__ eps, int *status) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double c_kms = 299792.458;
    const double arcsec_per_rad = 648000.0 / M_PI;
    double v = sigma[k] / c_kms;
    double ek = e[k];
    bool ok = (sigma[k] >= 0.0) && isfinite(sigma[k]) && (ek >= 0.0) && (ek < 1.0);
    b0[k] = ok ? K * M_PI * v * v * arcsec_per_rad : NAN;
    eps[k] = ok ? ek / (1.0 + sqrt(1.0 - ek * ek)) : NAN;
    if (!ok) atomicOr(status, ST_INVALID_TABLE);
}

hipError_t launch_phys_to_amp(const double *sigma, const double *e, int n, int convention,
                              double *b0, double *eps, int *status, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    double K = convention == 1 ? 4.0 : 6.0;
    hipLaunchKernelGGL(phys_to_amp_kernel, dim3((n + 255) / 256), dim3(256), 0, st, sigma, e, n, K,
                       b0, eps, status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Parameter prologue: amplitude-form table -> derived constants (FP64 block
// and, with F32, its FP32 copy; with LOG, the logarithmic term's constant).
template <bool F32, bool LOG>
__device__ __forceinline__ void prologue_one(const PotSoA &in, int k, double *__restrict__ dd,
                                             float *__restrict__ df, int stride, int *status) {
    prologue_values<F32, LOG>(in.x0[k], in.y0[k], in.b0[k], in.eps[k], in.phi[k], in.rcore[k],
                              in.rcut[k], k, dd, df, stride, status);
}

template <bool F32, bool LOG>
__global__ void prologue_kernel(PotSoA in, int n, double *__restrict__ dd, float *__restrict__ df,
                                int stride, int *status) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) prologue_one<F32, LOG>(in, k, dd, df, stride, status);
}

// Two tables in one launch (the fixed and the free potentials of a chi^2
// batch): threads [0, na) take table a, [na, na + nb) table b.
template <bool F32, bool LOG>
__global__ void prologue2_kernel(PotSoA a, int na, double *__restrict__ dda,
                                 float *__restrict__ dfa, int sa, PotSoA b, int nb,
                                 double *__restrict__ ddb, float *__restrict__ dfb, int sb,
                                 int *status) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < na)
        prologue_one<F32, LOG>(a, k, dda, dfa, sa, status);
    else if (k - na < nb)
        prologue_one<F32, LOG>(b, k - na, ddb, dfb, sb, status);
}

hipError_t launch_prologue2(PotSoA a, int na, double *dda, float *dfa, int sa, PotSoA b, int nb,
                            double *ddb, float *dfb, int sb, int *status, int parts,
                            hipStream_t st) {
    const long long n = (long long)na + nb;
    if (n <= 0) return hipSuccess;
    if (n > 0x7fffff00LL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    const bool f32 = parts & PRO_F32, lg = parts & PRO_LOG;
    if (f32 && lg)
        hipLaunchKernelGGL((prologue2_kernel<true, true>), grid, block, 0, st, a, na, dda, dfa,
                           sa, b, nb, ddb, dfb, sb, status);
    else if (f32)
        hipLaunchKernelGGL((prologue2_kernel<true, false>), grid, block, 0, st, a, na, dda, dfa,
                           sa, b, nb, ddb, dfb, sb, status);
    else if (lg)
        hipLaunchKernelGGL((prologue2_kernel<false, true>), grid, block, 0, st, a, na, dda, dfa,
                           sa, b, nb, ddb, dfb, sb, status);
    else
        hipLaunchKernelGGL((prologue2_kernel<false, false>), grid, block, 0, st, a, na, dda, dfa,
                           sa, b, nb, ddb, dfb, sb, status);
    return hipGetLastError();
}

hipError_t launch_prologue(PotSoA in, int n, double *dd, float *df, int stride, int *status,
                           int parts, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const dim3 grid((n + 255) / 256), block(256);
    const bool f32 = parts & PRO_F32, lg = parts & PRO_LOG;
    if (f32 && lg)
        hipLaunchKernelGGL((prologue_kernel<true, true>), grid, block, 0, st, in, n, dd, df,
                           stride, status);
    else if (f32)
        hipLaunchKernelGGL((prologue_kernel<true, false>), grid, block, 0, st, in, n, dd, df,
                           stride, status);
    else if (lg)
        hipLaunchKernelGGL((prologue_kernel<false, true>), grid, block, 0, st, in, n, dd, df,
                           stride, status);
    else
        hipLaunchKernelGGL((prologue_kernel<false, false>), grid, block, 0, st, in, n, dd, df,
                           stride, status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The map kernel.


// A wave-uniform double moved to scalar registers.
__device__ __forceinline__ double uniform_f64(double v) {
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                            __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
struct MapArgs {
    Derived tab;
    GridArgs g;
    double dlsds;
    void *out[5];
    void *dout[6];
    int derived;
    int chunk;
    Series S;
};

// Derived maps from the summed second derivatives h = (hxx, hxy, hyy) at one
// point (Sec. 2.4, Eqs. (7)-(9), with Sec. 2.1's inverse magnification matrix
// [[1 - kappa - gamma1, -gamma2], [-gamma2, 1 - kappa + gamma1]]):
// kappa, gamma1, gamma2, |gamma|, mu = 1/det, det = (1 - kappa)^2 - |gamma|^2.
__device__ __forceinline__ void derived_of(double hxx, double hxy, double hyy, double v[6]) {
    const double k = 0.5 * (hxx + hyy);
    const double g1 = 0.5 * (hxx - hyy);
    const double gg = g1 * g1 + hxy * hxy;
    const double om = 1.0 - k;
    const double det = om * om - gg;
    v[0] = k;
    v[1] = g1;
    v[2] = hxy;
    v[3] = sqrt(gg);
    v[4] = 1.0 / det;
    v[5] = det;
}

// Minimum waves per SIMD the register allocation must allow: the FP64 kernel
// with one pixel per thread fits six without spilling (80 registers); the
// other variants keep the compiler's choice.
template <int PREC, int PPT>
constexpr int map_min_waves() {
    return (PREC == 0 && PPT == 1) ? 6 : 1;
}

template <int PREC, bool GRAD, bool HESS, bool STAGE, int PPT>
__global__ void __launch_bounds__(256, (map_min_waves<PREC, PPT>())) map_kernel(MapArgs a) {
    extern __shared__ double lds[];
    const int bx = blockDim.x, by = blockDim.y;
    const int i_base = blockIdx.x * bx * PPT + threadIdx.x;
    // block_x is a multiple of 64, so a wave never spans two rows: the row
    // index and its coordinate are wave-uniform and live in scalar registers
    const int j = __builtin_amdgcn_readfirstlane(blockIdx.y * by + threadIdx.y);
    const double y = uniform_f64(grid_coord(a.g.y0, j, a.g.dy));
    double x[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) x[p] = grid_coord(a.g.x0, i_base + p * bx, a.g.dx);

    // accumulators: FP64 (PREC 0, 1) or compensated FP32 (PREC 2)
    double acc[PPT][5];
    float fs[PPT][5], fc[PPT][5];
#pragma unroll
    for (int p = 0; p < PPT; ++p)
#pragma unroll
        for (int ch = 0; ch < 5; ++ch) {
            acc[p][ch] = 0.0;
            fs[p][ch] = 0.f;
            fc[p][ch] = 0.f;
        }

    const int n = a.tab.n, st = a.tab.stride;
    // The polynomials' first step multiplies the leading coefficient and adds
    // the next: with both in scalar registers every evaluation would copy one
    // to a vector register first (one constant-bus operand per instruction),
    // so the leading coefficients are held in vector registers for the loop.
    Series S = a.S;
    if (PREC == 0) {
        S.at[0] = vgpr_f64(a.S.at[0]);
        S.ah[0] = vgpr_f64(a.S.ah[0]);
        S.ats[0] = vgpr_f64(a.S.ats[0]);
        S.ahs[0] = vgpr_f64(a.S.ahs[0]);
    }
    // one potential (kind: its wave-uniform kind bits) at the thread's pixels;
    // they share the row, so dy and its rotated parts are formed once
    auto body = [&](const ConstD cd, const ConstF cf, int kind) {
        if (PREC == 0) {
            const double dy = y - cd[D_Y0];
            const double dyc = dy * cd[D_C], dys = dy * cd[D_S], x0 = cd[D_X0];
#pragma unroll
            for (int p = 0; p < PPT; ++p)
                eval_pot_f64_rel<GRAD, HESS, true>(cd, kind, x[p] - x0, dy, dyc, dys, acc[p], S);
            return;
        }
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            float o[5];
            eval_pot_f32_kind<GRAD, HESS, true>(cd, cf, kind, x[p], y, o, a.S);
#pragma unroll
            for (int ch = 0; ch < 5; ++ch) {
                const bool used = (ch < 2) ? GRAD : HESS;
                if (!used) continue;
                if (PREC == 1)
                    acc[p][ch] += (double)o[ch];
                else
                    neumaier_add(fs[p][ch], fc[p][ch], o[ch]);
            }
        }
    };

    if (STAGE) {
        const int chunk = a.chunk;
        // waves of the block (block_x is a multiple of 64) and lane in the wave
        const int tid = threadIdx.y * bx + threadIdx.x;
        const int wv = tid >> 6, lane = tid & 63, nw = (bx * by) >> 6;
        float *ldsf = reinterpret_cast<float *>(lds + (size_t)chunk * NDER);
        for (int k0 = 0; k0 < n; k0 += chunk) {
            const int cnt = min(chunk, n - k0);
            __syncthreads();
            // wave wv copies the constants wv, wv + nw, ... of the chunk's
            // potentials, its lanes consecutive potentials (coalesced reads),
            // four constants' loads in flight before their LDS writes
            for (int kk = lane; kk < cnt; kk += 64) {
                for (int c0 = wv; c0 < NDER; c0 += 4 * nw) {
                    double v[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int ci = c0 + u * nw;
                        v[u] = ci < NDER ? a.tab.d[(size_t)ci * st + k0 + kk] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int ci = c0 + u * nw;
                        if (ci < NDER) lds[kk * NDER + ci] = v[u];
                    }
                }
                if (PREC != 0) {
                    for (int c0 = wv; c0 < NDERF; c0 += 4 * nw) {
                        float v[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int ci = c0 + u * nw;
                            v[u] = ci < NDERF ? a.tab.f[(size_t)ci * st + k0 + kk] : 0.f;
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int ci = c0 + u * nw;
                            if (ci < NDERF) ldsf[kk * NDERF + ci] = v[u];
                        }
                    }
                }
            }
            __syncthreads();
            for (int kb = 0; kb < cnt; kb += 64) {
                // the kinds of the next (up to) 64 potentials as one bit mask
                // per kind bit (lane l reads potential kb + l), so that the
                // loop takes each potential's kind in scalar registers
                const int m = min(64, cnt - kb);
                const KindMasks km =
                    kind_masks(lane < m ? kind_bits(lds[(kb + lane) * NDER + D_KIND]) : 0);
                const double *row = lds_entry(lds, kb * NDER);
                for (int i = 0; i < m; ++i)
                    body(ConstD{row + i * NDER, 1}, ConstF{ldsf + (kb + i) * NDERF, 1},
                         km.kind(i));
            }
        }
    } else {
        for (int k = 0; k < n; ++k)
            body(ConstD{a.tab.d + k, st}, ConstF{a.tab.f + k, st},
                 uniform_kind(a.tab.d[(size_t)D_KIND * st + k]));
    }

    if (j >= a.g.ny) return;
    // summed values per channel: deflection, then psi_xx, psi_xy, psi_yy from
    // the accumulated trace, difference and off-diagonal parts
    double tot[PPT][5];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
#pragma unroll
        for (int ch = 0; ch < 5; ++ch)
            tot[p][ch] = PREC == 2 ? (double)fs[p][ch] + (double)fc[p][ch] : acc[p][ch];
        if (HESS) hess_of_parts(tot[p][2], tot[p][3], tot[p][4], &tot[p][2]);
    }
    if (HESS && a.derived) {
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int i = i_base + p * bx;
            if (i >= a.g.nx) continue;
            const size_t idx = (size_t)j * a.g.nx + i;
            double h[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) h[c] = a.dlsds * tot[p][2 + c];
            double v[6];
            derived_of(h[0], h[1], h[2], v);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                if (a.dout[c] == nullptr) continue;
                if (PREC == 0)
                    static_cast<double *>(a.dout[c])[idx] = v[c];
                else
                    static_cast<float *>(a.dout[c])[idx] = (float)v[c];
            }
        }
        return;
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int i = i_base + p * bx;
        if (i >= a.g.nx) continue;
        const size_t idx = (size_t)j * a.g.nx + i;
#pragma unroll
        for (int ch = 0; ch < 5; ++ch) {
            if (a.out[ch] == nullptr) continue;
            if (PREC == 0)
                static_cast<double *>(a.out[ch])[idx] = a.dlsds * tot[p][ch];
            else
                static_cast<float *>(a.out[ch])[idx] = (float)(a.dlsds * tot[p][ch]);
        }
    }
}

typedef void (*MapKernelFn)(MapArgs);

template <int PREC, bool GRAD, bool HESS>
static MapKernelFn pick_ppt(bool stage, int ppt) {
    if (stage) {
        if (ppt == 1) return map_kernel<PREC, GRAD, HESS, true, 1>;
        if (ppt == 2) return map_kernel<PREC, GRAD, HESS, true, 2>;
    } else {
        if (ppt == 1) return map_kernel<PREC, GRAD, HESS, false, 1>;
        if (ppt == 2) return map_kernel<PREC, GRAD, HESS, false, 2>;
    }
    return nullptr;
}

template <int PREC>
static MapKernelFn pick_mode(bool grad, bool hess, bool stage, int ppt) {
    if (grad && hess) return pick_ppt<PREC, true, true>(stage, ppt);
    if (grad) return pick_ppt<PREC, true, false>(stage, ppt);
    if (hess) return pick_ppt<PREC, false, true>(stage, ppt);
    return nullptr;
}

bool map_tuning_valid(const lens_map_tuning_t &t) {
    if (t.block_x <= 0 || t.block_x % 64 != 0 || t.block_y <= 0) return false;
    if ((long long)t.block_x * t.block_y > 256) return false;
    if (t.pix_per_thread != 1 && t.pix_per_thread != 2) return false;
    if (t.stage != 0 && t.stage != 1) return false;
    if (t.stage == 1 && (t.lds_chunk < 1 || t.lds_chunk > 256)) return false;
    return true;
}

hipError_t launch_map(const MapLaunch &m, hipStream_t st) {
    const lens_map_tuning_t &t = m.tune;
    MapKernelFn fn = nullptr;
    const bool stage = t.stage == 1;
    if (m.prec == 0) fn = pick_mode<0>(m.grad, m.hess, stage, t.pix_per_thread);
    if (m.prec == 1) fn = pick_mode<1>(m.grad, m.hess, stage, t.pix_per_thread);
    if (m.prec == 2) fn = pick_mode<2>(m.grad, m.hess, stage, t.pix_per_thread);
    if (!fn) return hipErrorInvalidValue;
    MapArgs a;
    a.tab = m.tab;
    a.g = m.grid;
    a.dlsds = m.dlsds;
    for (int c = 0; c < 5; ++c) a.out[c] = m.out[c];
    for (int c = 0; c < 6; ++c) a.dout[c] = m.derived ? m.dout[c] : nullptr;
    a.derived = m.derived ? 1 : 0;
    if (m.derived && !m.hess) return hipErrorInvalidValue;
    a.chunk = t.lds_chunk;
    a.S = make_series();
    const long long span_x = (long long)t.block_x * t.pix_per_thread;
    dim3 grid((unsigned)((m.grid.nx + span_x - 1) / span_x),
              (unsigned)((m.grid.ny + t.block_y - 1) / t.block_y));
    if (grid.y > 65535u) return hipErrorInvalidConfiguration;
    dim3 block(t.block_x, t.block_y);
    size_t shmem = 0;
    if (stage) shmem = (size_t)t.lds_chunk * (NDER * sizeof(double) + NDERF * sizeof(float));
    hipLaunchKernelGGL(fn, grid, block, shmem, st, a);
    return hipGetLastError();
}

}  // namespace lens
