// potential.hip -- lensing potential and time-delay maps (Sec. 2.4 names the
// potential and the time-delay surface among the lensing maps; alpha = grad
// psi, Sec. 2.1).
//
// Each cored isothermal ellipsoid contributes (Keeton 2001, softened
// isothermal ellipsoid, under the mapping b = b0(1+eps), q = (1-eps)/(1+eps),
// s_K = (1+eps) w of the deflection)
//   P_w = x' a'x,w + y' a'y,w - L_w ln D_w / 2,
//   D_w = (psi_w + S_w)^2 + k^2 x'^2,  L_w = b0 (1 - eps^2) w,
// (circular: D_w = (psi_w + w)^2), and a dPIE F (P_a - P_s).  The two cores'
// deflection terms combine as in the deflection map (one atan and one atanh
// per potential); x' a'x + y' a'y is a dot product, so no rotation back is
// needed.  L_w = PF k S_w (elliptical) or PF S_w (circular) in terms of the
// derived constants, PF including F (PF k = F b0 (1 - eps)).
//
// Design (gfx950): one thread per pixel, the potentials staged in LDS in
// chunks and read by broadcast (as in the deflection map), FP64 throughout.
#include <math.h>

#include "eval.h"
#include "potential_launch.h"

namespace lens {

// ln D for D > 0: D = m 2^e with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s),
// s = (m - 1)/(m + 1) (|s| <= 3 - 2 sqrt 2), by the atanh polynomial of eval.h.
// Split in two so that the reciprocal of m + 1 can be shared with others.
struct LogRed {
    double m;  // mantissa in [sqrt(1/2), sqrt(2))
    int e;
};
__device__ __forceinline__ LogRed log_reduce(double D) {
    LogRed r;
    r.m = __builtin_amdgcn_frexp_mant(D);  // [0.5, 1)
    r.e = __builtin_amdgcn_frexp_exp(D);
    if (r.m < 0.7071067811865476) {
        r.m = 2.0 * r.m;
        r.e -= 1;
    }
    return r;
}
__device__ __forceinline__ double log_finish(const LogRed &r, double inv_m1, const Series &S) {
    const double s = (r.m - 1.0) * inv_m1;
    const double s2 = s * s;
    double p = S.ah[0];
#pragma unroll
    for (int i = 1; i < LENS_ATANH_N; ++i) p = fma(p, s2, S.ah[i]);
    const double t = fma(s * s2, p, s);
    return fma(kLn2, (double)r.e, 2.0 * t);
}
__device__ __forceinline__ double log_pos(double D, const Series &S) {
    const LogRed r = log_reduce(D);
    return log_finish(r, rcp64(r.m + 1.0), S);
}

// Potential of one potential at (x, y), Dls/Ds = 1.
__device__ __forceinline__ double eval_psi_f64(const ConstD c, double x, double y,
                                               const Series &S) {
    const int kind = uniform_kind(c[D_KIND]);
    double dx = x - c[D_X0];
    double dy = y - c[D_Y0];
    bool zero = false;
    if (kind & K_SING) {
        zero = (dx == 0.0) & (dy == 0.0);
        if (zero) dx = 1.0;  // any regular point; the contribution is dropped
    }
    const double cp = c[D_C], sp = c[D_S];
    const double xp = fma(dx, cp, dy * sp);
    const double yp = fma(-sp, dx, dy * cp);
    const double x2 = xp * xp, y2 = yp * yp;
    double v = 0.0;
    // Elliptical forms in the lengths divided by k, as in the deflection map:
    // the log terms' D_w/k^2 leave the constant L_w ln(k) per core, carried
    // with the log terms' factors in D_LA, D_LS, D_LC.
    switch (kind & (K_CUT | K_ELL)) {
    case K_CUT | K_ELL: {
        const double ta = fma(c[D_EQ2], x2, fma(c[D_EK2I], y2, c[D_ECA]));
        const double ts = ta + c[D_DC];
        const double ra = rsq2q(ta), rs = rsq2q(ts);  // quarter radii, as in the map
        const double A1 = fma(ta, ra, c[D_ESA]), A2 = fma(ts, rs, c[D_ESS]);
        const double B1 = fma(ta, ra, c[D_EQ2SA]), B2 = fma(ts, rs, c[D_EQ2SS]);
        const double Dx = fma(A1, A2, x2);
        const double Dy = fma(B1, B2, -y2);
        // the log terms' mantissas, then one reciprocal (a quarter-rate
        // instruction) for 1/(Dx Dy) and the two 1/(m + 1)
        const LogRed lra = log_reduce(fma(A1, A1, x2)), lrs = log_reduce(fma(A2, A2, x2));
        const double DXY = Dx * Dy;
        const double ma1 = lra.m + 1.0, ms1 = lrs.m + 1.0, M = ma1 * ms1;
        const double Rr = rcp64(DXY * M);
        const double RM = Rr * M, RP = Rr * DXY;  // 1/(Dx Dy), 1/M
        const double Nx = xp * (A2 - A1);
        const double Ny = yp * (B2 - B1);
        // the deflection's two fast tiers (small ratios on the whole wave), as
        // in the deflection map
        const double bf = Nx * (RM * Dy), sf = Ny * (RM * Dx);
        double tx = atan_poly_s(bf, S), ty = atanh_poly_s(sf, S);
        if (!wave_all(fabs(bf) <= kAtanSMax, fabs(sf) <= kAtanhSMax)) {
            if (wave_all(fabs(bf) <= kTanPi16, fabs(sf) <= kAtanhS)) {
                tx = atan_poly(bf, S);
                ty = atanh_poly(sf, S);
            } else {
                const AtanRed ra_ = atan_reduce(Nx, Dx);
                const AtanhRed rh = atanh_reduce(Ny, Dy);
                const double R2 = rcp64(ra_.den * rh.den);
                tx = atan_finish(ra_, ra_.num * (R2 * rh.den), S);
                ty = atanh_finish(rh, rh.num * (R2 * ra_.den), S);
            }
        }
        const double ax = c[D_PF] * tx, ay = c[D_PF] * ty;
        const double la = log_finish(lra, RP * ms1, S), ls = log_finish(lrs, RP * ma1, S);
        const double L = fma(c[D_LA], la, fma(-c[D_LS], ls, c[D_LC]));
        v = fma(xp, ax, yp * ay) - L;
        break;
    }
    case K_CUT: {
        const double R = fma(c[D_Q2], x2, y2);
        const double ta = c[D_CA] + R, ts = c[D_CS_] + R;
        const double pa = ta * rsq64(ta), ps = ts * rsq64(ts);
        const double A1 = pa + c[D_SA], A2 = ps + c[D_SS];
        const double sum = pa + ps;
        const double A12 = A1 * A2;
        const double R1 = rcp64(sum * A12);
        const double g = c[D_DC] * (R1 * A12);
        const double t = c[D_PF] * (g + c[D_DS]) * (R1 * sum);
        const double L = c[D_PF] * (c[D_SA] * log_pos(A1, S) - c[D_SS] * log_pos(A2, S));
        v = t * (x2 + y2) - L;
        break;
    }
    case K_ELL: {
        const double ta = fma(c[D_EQ2], x2, fma(c[D_EK2I], y2, c[D_ECA]));
        const double ra = rsq2q(ta);
        const double A1 = fma(ta, ra, c[D_ESA]);
        const double B1 = fma(ta, ra, c[D_EQ2SA]);
        const AtanRed ra_ = atan_reduce(xp, A1);
        const AtanhRed rh = atanh_reduce(yp, B1);
        const double R2 = rcp64(ra_.den * rh.den);
        const double ax = c[D_PF] * atan_finish(ra_, ra_.num * (R2 * rh.den), S);
        const double ay = c[D_PF] * atanh_finish(rh, rh.num * (R2 * ra_.den), S);
        const double L = fma(c[D_LA], log_pos(fma(A1, A1, x2), S), c[D_LC]);
        v = fma(xp, ax, yp * ay) - L;
        break;
    }
    default: {
        const double ta = c[D_CA] + fma(c[D_Q2], x2, y2);
        const double A1 = ta * rsq64(ta) + c[D_SA];
        const double t = c[D_PF] * rcp64(A1);
        const double L = c[D_SA] == 0.0 ? 0.0 : c[D_PF] * (c[D_SA] * log_pos(A1, S));
        v = t * (x2 + y2) - L;
        break;
    }
    }
    return zero ? 0.0 : v;
}

struct PotMapArgs {
    Derived tab;
    GridArgs g;
    double dlsds, bx, by, scale;
    double *out;
    int td;  // 1: time-delay surface scale (|theta - beta|^2/2 - psi)
    Series S;
};

constexpr int PSI_CHUNK = 64;

__global__ void __launch_bounds__(256) potential_map_kernel(PotMapArgs a) {
    __shared__ double pd[PSI_CHUNK * NDER];
    const int tid = threadIdx.y * 64 + threadIdx.x;
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    const double x = grid_coord(a.g.x0, i, a.g.dx);
    const double y = grid_coord(a.g.y0, j, a.g.dy);
    const int n = a.tab.n, st = a.tab.stride;
    double acc = 0.0;
    for (int k0 = 0; k0 < n; k0 += PSI_CHUNK) {
        const int cnt = min(PSI_CHUNK, n - k0);
        __syncthreads();
        for (int e = tid; e < cnt * NDER; e += 256) {
            const int ci = e / cnt, kk = e - ci * cnt;
            pd[kk * NDER + ci] = a.tab.d[(size_t)ci * st + k0 + kk];
        }
        __syncthreads();
        for (int kk = 0; kk < cnt; ++kk) acc += eval_psi_f64(ConstD{pd + kk * NDER, 1}, x, y, a.S);
    }
    if (i >= a.g.nx || j >= a.g.ny) return;
    const size_t idx = (size_t)j * a.g.nx + i;
    if (a.td) {
        const double ex = x - a.bx, ey = y - a.by;
        a.out[idx] = a.scale * (0.5 * (ex * ex + ey * ey) - a.dlsds * acc);
    } else {
        a.out[idx] = a.dlsds * acc;
    }
}

hipError_t launch_potential_map(Derived tab, GridArgs g, double dlsds, double *out, int td,
                                double bx, double by, double scale, hipStream_t st) {
    if (g.nx <= 0 || g.ny <= 0) return hipSuccess;
    PotMapArgs a;
    a.tab = tab;
    a.g = g;
    a.dlsds = dlsds;
    a.bx = bx;
    a.by = by;
    a.scale = scale;
    a.out = out;
    a.td = td;
    a.S = make_series();
    dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + 3) / 4));
    if (grid.y > 65535u) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(potential_map_kernel, grid, dim3(64, 4), 0, st, a);
    return hipGetLastError();
}

}  // namespace lens
