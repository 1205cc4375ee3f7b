// eval.h -- per-potential deflection / second-derivative evaluation on gfx950.
//
// One call evaluates one potential at one point and adds its contribution to
// the accumulators.  On the hot paths every lane of a wave evaluates the same
// potential at the same time, so the branches on the potential's kind are
// uniform across the wave (the kind is read into a scalar register).
//
// Math (Keeton 2001 closed forms of the cored isothermal ellipsoid, mapped to
// the Kassiola-Kovner ellipticity of the dPIE; the paper's Sec. 2.2 model
// parameters, summed per Sec. 4.1 Eq. (10) and Sec. 2.4 Eqs. (7)-(9)):
//   two cores a < s combine as F (P_a - P_s); the arctangent and hyperbolic
//   arctangent differences use
//     atan(kx/A_a) - atan(kx/A_s)   = atan(k x (A_s - A_a) / (A_a A_s + k^2 x^2))
//     atanh(ky/B_a) - atanh(ky/B_s) = atanh(k y (B_s - B_a) / (B_a B_s - k^2 y^2))
//   (both arguments have the same sign, so no branch correction is needed).
//   A_s - A_a = (C_s - C_a)/(psi_a + psi_s) + (S_s - S_a), which does not cancel.
//
// Arithmetic (FP64 path).  The accuracy target is a few units in the last
// place, far inside the 1e-12 relative tolerance of the map, so the path uses
// no correctly-rounded division or square root:
//   - 1/sqrt(x) and 1/x start from the hardware estimates (v_rsq_f64,
//     v_rcp_f64) and take one Newton step each;
//   - reciprocals needed at the same time share one reciprocal of their
//     product (1/a = b/(ab), 1/b = a/(ab));
//   - atan(N/D) is reduced to |b| <= tan(pi/16) with atan(t) = pi/2 -
//     atan(1/t) and a shift to the nearest of three centres, then
//     atan(b) = b + b^3 p(b^2) with p of degree 7 (a Chebyshev interpolant;
//     relative error below 1e-18 with its FP64 coefficients);
//   - atanh(N/D) = ln(P/Q)/2, P = D + N, Q = D - N, is reduced by the binary
//     exponent k of P/Q to ln(P/Q) = k ln 2 + 2 atanh(s), s = (P 2^-k - Q) /
//     (P 2^-k + Q) (s = N/D exactly when k = 0), |s| <= 3 - 2 sqrt(2), and
//     atanh(s) = s + s^3 q(s^2) with q of degree 6 (relative error below
//     5e-18).
#pragma once

#include "lens_internal.h"

namespace lens {

// Constants of one potential, read through an accessor: AoS in LDS
// (stride 1) or the SoA table in global memory (stride = table stride).
struct ConstD {
    const double *p;
    int st;
    __device__ __forceinline__ double operator[](int i) const { return p[i * st]; }
};
struct ConstF {
    const float *p;
    int st;
    __device__ __forceinline__ float operator[](int i) const { return p[i * st]; }
};

// The kind bits are the low word of the D_KIND entry's bit pattern (no
// conversion instruction; read into a scalar register on the uniform path).
__device__ __forceinline__ int kind_bits(double k) { return __double2loint(k); }
__device__ __forceinline__ int uniform_kind(double k) {
    return __builtin_amdgcn_readfirstlane(__double2loint(k));
}

// A copy of a double in vector registers (kept there: the compiler cannot
// rematerialise it from the scalar source).
__device__ __forceinline__ double vgpr_f64(double x) {
    double r;
    asm volatile("v_mov_b64 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

// &base[off] for a wave-uniform off, the address held in a vector register:
// entries addressed from it are read with one vector add for their address
// (left to itself the compiler keeps a uniform address in a scalar register
// and copies it to a vector register before each group of reads).
__device__ __forceinline__ const double *lds_entry(const double *base, int off) {
    int v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(off * (int)sizeof(double)));
    return reinterpret_cast<const double *>(reinterpret_cast<const char *>(base) + v);
}

// The kinds of up to 64 staged potentials as one bit mask per kind bit (lane
// l of the wave reads entry l; the caller's whole wave is active), and the
// kind of entry i from the masks with scalar operations: a loop over staged
// potentials then takes each one's kind without a copy from a vector
// register.
struct KindMasks {
    unsigned long long ell, cut, sing, e32;
    __device__ __forceinline__ int kind(int i) const {
        return (int)((ell >> i) & 1) * K_ELL | (int)((cut >> i) & 1) * K_CUT |
               (int)((sing >> i) & 1) * K_SING | (int)((e32 >> i) & 1) * K_ELL32;
    }
};
__device__ __forceinline__ KindMasks kind_masks(int kl) {
    KindMasks m;
    m.ell = __builtin_amdgcn_ballot_w64(kl & K_ELL);
    m.cut = __builtin_amdgcn_ballot_w64(kl & K_CUT);
    m.sing = __builtin_amdgcn_ballot_w64(kl & K_SING);
    m.e32 = __builtin_amdgcn_ballot_w64(kl & K_ELL32);
    return m;
}

// True on every active lane when both predicates hold on all of them (scalar
// operations on the compare masks and the execution mask).
__device__ __forceinline__ bool wave_all(bool p, bool q) {
    return (__builtin_amdgcn_ballot_w64(p) & __builtin_amdgcn_ballot_w64(q)) ==
           __builtin_amdgcn_read_exec();
}

// ---------------------------------------------------------------------------
// FP64 building blocks
// The hardware estimates are accurate to about 2^-24 (measured over 2^20
// inputs spanning 2^-30..2^30); one Newton step brings the reciprocal to
// 2.2e-15 and the reciprocal square root to 4.1e-15 relative error.
__device__ __forceinline__ double rcp64(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(fma(-x, r, 1.0), r, r);
}

__device__ __forceinline__ double rsq64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return fma(y, fma(-0.5 * x, y * y, 0.5), y);
}

// 2/sqrt(T) from the estimate w by the same Newton step written as
// w (3 - T w^2) (three instructions: the halving of the step is left in the
// result).  The elliptical forms hold T = R/4, a quarter of the squared
// radius R = psi^2/k^2, so this is 4/sqrt(R), and T times it is sqrt(R).
// Relative error: about 1.5 times the square of the estimate's plus three
// roundings (4.5e-15 at most over the measured estimate range).
__device__ __forceinline__ double rsq2q(double T) {
    const double w = __builtin_amdgcn_rsq(T);
    return w * fma(-T, w * w, 3.0);
}

constexpr double kPi2 = 1.5707963267948966;
constexpr double kPi4 = 0.7853981633974483;
constexpr double kLn2 = 0.6931471805599453;

// atan(N/D), D > 0: t = min/max of |N|, D in [0, 1] is shifted to the
// nearest of the centres c = 0, tan(pi/8), 1 by atan(t) = atan(c) +
// atan((t - c)/(1 + t c)) (exact for the rounded centre, whose arctangent is
// the stored constant), leaving |b| <= tan(pi/16); then atan(|N|/D) =
// pi/2 - atan(D/|N|) when |N| > D.  Then the polynomial of degree 7 in b^2.
constexpr double kTanPi16 = 0.198912367379658;
constexpr double kTan3Pi16 = 0.6681786379192989;
constexpr double kC1 = 0.41421356237309503;       // tan(pi/8), rounded
constexpr double kAtanC1 = 0.39269908169872414;   // atan of the rounded value
struct AtanRed {
    double num, den, base;
    bool big;
    double sign;
};
__device__ __forceinline__ AtanRed atan_reduce(double N, double D) {
    const double u = fabs(N);
    const bool big = u > D;
    const double lo = fmin(u, D), hi = fmax(u, D);  // (finite operands)
    const bool m1 = lo > kTanPi16 * hi, m2 = lo > kTan3Pi16 * hi;
    const double c = m2 ? 1.0 : (m1 ? kC1 : 0.0);
    AtanRed r;
    r.num = fma(-c, hi, lo);
    r.den = fma(c, lo, hi);
    r.base = m2 ? kPi4 : (m1 ? kAtanC1 : 0.0);
    r.big = big;
    r.sign = N;
    return r;
}
// atan(b) for |b| <= tan(pi/16): b + b^3 p(b^2).
__device__ __forceinline__ double atan_poly(double b, const Series &S) {
    const double b2 = b * b;
    double p = S.at[0];
#pragma unroll
    for (int i = 1; i < LENS_ATAN_N; ++i) p = fma(p, b2, S.at[i]);
    return fma(b * b2, p, b);
}
// The same on |b| <= tan(pi/16)/5 with the shorter polynomial.
constexpr double kAtanSMax = LENS_ATAN_S_MAX;
__device__ __forceinline__ double atan_poly_s(double b, const Series &S) {
    const double b2 = b * b;
    double p = S.ats[0];
#pragma unroll
    for (int i = 1; i < LENS_ATAN_S_N; ++i) p = fma(p, b2, S.ats[i]);
    return fma(b * b2, p, b);
}
__device__ __forceinline__ double atan_finish(const AtanRed &r, double b, const Series &S) {
    double t = atan_poly(b, S) + r.base;
    t = r.big ? kPi2 - t : t;
    return copysign(t, r.sign);
}

// atanh(N/D) for |N| < D: reduction of ln((D+N)/(D-N)).
struct AtanhRed {
    double num, den;
    int k;
};
__device__ __forceinline__ AtanhRed atanh_reduce(double N, double D) {
    const double P = D + N, Q = D - N;
    // k ~ log2(P/Q) from the two positive operands' high words (exponent and
    // the first 20 mantissa bits: log2(1 + m) read as m), rounded: the reduced
    // ratio P 2^-k / Q is within 2^(1/2 + 0.0861) of 1 and the quotient below
    // within LENS_ATANH_R_MAX, the interval of the polynomial
    int k = (__double2hiint(P) - __double2hiint(Q) + (1 << 19)) >> 20;
    // (an empty statement fixes k here: moved earlier by the scheduler, the
    // two interleaved points' reductions needed five more registers and the
    // source-plane kernels spilled)
    asm volatile("" : "+v"(k));
    // (D+N) 2^-k - (D-N) as (D+N)(2^-k - 1) + 2N: exactly 2N when k = 0, with
    // no select; 2^-k - 1 is exact for the exponents that occur
    const double t = __builtin_amdgcn_ldexp(1.0, -k);
    AtanhRed r;
    r.num = fma(P, t - 1.0, 2.0 * N);
    r.den = fma(P, t, Q);
    r.k = k;
    return r;
}
// atanh(s) for |s| <= LENS_ATANH_R_MAX (0.2004, what the reduction leaves):
// s + s^3 q(s^2).  The first polynomial tier takes the narrower 3 - 2 sqrt 2.
constexpr double kAtanhS = 0.171572875253809;  // 3 - 2 sqrt 2, rounded down
__device__ __forceinline__ double atanh_poly(double s, const Series &S) {
    const double s2 = s * s;
    double p = S.ah[0];
#pragma unroll
    for (int i = 1; i < LENS_ATANH_N; ++i) p = fma(p, s2, S.ah[i]);
    return fma(s * s2, p, s);
}
// The same on |s| <= (3 - 2 sqrt 2)/5 with the shorter polynomial.
constexpr double kAtanhSMax = LENS_ATANH_S_MAX;
__device__ __forceinline__ double atanh_poly_s(double s, const Series &S) {
    const double s2 = s * s;
    double p = S.ahs[0];
#pragma unroll
    for (int i = 1; i < LENS_ATANH_S_N; ++i) p = fma(p, s2, S.ahs[i]);
    return fma(s * s2, p, s);
}
__device__ __forceinline__ double atanh_finish(const AtanhRed &r, double s, const Series &S) {
    return fma(0.5 * kLn2, (double)r.k, atanh_poly(s, S));
}

// ---------------------------------------------------------------------------
// A potential with rcore = 0 (K_SING) contributes zero at its own centre
// (where the closed forms give NaN): one block at the end, guarded by the kind
// bit, after the body that every kind shares (on a wave-uniform kind a scalar
// branch that regular potentials skip; the accumulators stay in one set of
// registers).
//
// The point enters as its offsets (dx, dy) from the centre with dy cos(phi) and
// dy sin(phi) (dyc, dys): a caller whose points share a row forms the last two
// once per potential.
template <bool GRAD, bool HESS, bool SHORT>
__device__ __forceinline__ void eval_pot_f64_impl(const ConstD c, int kind, double dx, double dy,
                                                  double dyc, double dys, double acc[5],
                                                  const Series &S) {
    const double cp = c[D_C], sp = c[D_S];
    const double xp = fma(dx, cp, dys);
    const double yp = fma(-sp, dx, dyc);
    const double x2 = xp * xp, y2 = yp * yp;
    // htr, hdf: psi_xx + psi_yy and psi_xx - psi_yy; hxy holds -psi_xy
    double ax = 0.0, ay = 0.0, htr = 0.0, hdf = 0.0, hxy = 0.0;
    // Two cores (ra, rs: 1/psi_w up to the form's constant factor; iDa, iDs:
    // 1/D_w): trace r_a - r_s, and the difference and -psi_xy from
    // h_w = 1/(psi_w D_w).
    const auto hess2 = [&](double ra, double rs, double iDa, double iDs) {
        const double ha = ra * iDa, hs = rs * iDs;
        const double dh = ha - hs;
        htr = ra - rs;
        hdf = fma(y2 - x2, dh, fma(ha, c[D_EA], -(hs * c[D_ES])));
        hxy = (xp * yp) * dh;
    };
    const auto hess1 = [&](double ra, double iDa) {
        const double ha = ra * iDa;
        htr = ra;
        hdf = ha * ((y2 - x2) + c[D_EA]);
        hxy = (xp * yp) * ha;
    };
    // The four forms by a scalar switch on the kind bits, so that no kind test
    // is carried from one form's code into another's.  Elliptical potentials
    // work with every length of the closed form divided by k (psi_w/k, A_w/k,
    // B_w/k): the ratios k x'/A_w and k y'/B_w lose their k and D_w/k^2 =
    // A_w^2/k^2 + x'^2; the Hessian constants carry the factors k and 1/k^3
    // this leaves on the trace and on the other parts, and the factor 1/4 of
    // ra, rs = 4 k/psi_w (from rsq2q of the quarter radii ta, ts).
    switch (kind & (K_CUT | K_ELL)) {
    case K_CUT | K_ELL: {
        // psi_w^2/(4 k^2), the second as the first plus (C_s - C_a)/(4 k^2);
        // psi_w/k = ta ra enters A_w/k and B_w/k through one FMA each
        const double ta = fma(c[D_EQ2], x2, fma(c[D_EK2I], y2, c[D_ECA]));
        const double ts = ta + c[D_DC];
        const double ra = rsq2q(ta), rs = rsq2q(ts);
        const double A1 = fma(ta, ra, c[D_ESA]), A2 = fma(ts, rs, c[D_ESS]);
        // one reciprocal (a quarter-rate instruction) of D_a D_s Dx Dy serves
        // the Hessian denominators and the ratios' denominators Dx = A_a A_s +
        // x'^2 and Dy = B_a B_s - y'^2 (the two cores' arctangents and
        // hyperbolic arctangents subtracted in closed form)
        double Da = 1.0, Ds = 1.0, DD = 1.0, iDa = 0.0, iDs = 0.0;
        if (HESS) {
            Da = fma(A1, A1, x2);
            Ds = fma(A2, A2, x2);
            DD = Da * Ds;
        }
        if (GRAD) {
            const double B1 = fma(ta, ra, c[D_EQ2SA]), B2 = fma(ts, rs, c[D_EQ2SS]);
            const double Dx = fma(A1, A2, x2);
            const double Dy = fma(B1, B2, -y2);
            const double XG = Dx * Dy;
            const double Rall = rcp64(HESS ? DD * XG : XG);
            if (HESS) {
                const double t = Rall * XG;  // 1/(D_a D_s)
                iDa = t * Ds;
                iDs = t * Da;
            }
            const double R2 = HESS ? Rall * DD : Rall;  // 1/(Dx Dy)
            const double Nx = xp * (A2 - A1);
            const double Ny = yp * (B2 - B1);
            // Away from the cores both ratios are small: when they are inside
            // the polynomials' intervals for the whole wave, the reductions
            // are skipped, and (SHORT) when they are inside the first fifth
            // of them, the shorter polynomials serve.  (The polynomials are
            // evaluated before the tests, into the registers the results
            // keep; the waves that fail a test overwrite them.)
            const double bf = Nx * (R2 * Dy), sf = Ny * (R2 * Dx);
            if (SHORT) {
                ax = atan_poly_s(bf, S);
                ay = atanh_poly_s(sf, S);
            }
            if (!SHORT || !wave_all(fabs(bf) <= kAtanSMax, fabs(sf) <= kAtanhSMax)) {
                ax = atan_poly(bf, S);
                ay = atanh_poly(sf, S);
                if (!wave_all(fabs(bf) <= kTanPi16, fabs(sf) <= kAtanhS)) {
                    const AtanRed ra_ = atan_reduce(Nx, Dx);
                    const AtanhRed rh = atanh_reduce(Ny, Dy);
                    const double R3 = rcp64(ra_.den * rh.den);
                    const double b = ra_.num * (R3 * rh.den);
                    const double s = rh.num * (R3 * ra_.den);
                    ax = atan_finish(ra_, b, S);
                    ay = atanh_finish(rh, s, S);
                }
            }
        } else if (HESS) {
            const double t = rcp64(DD);
            iDa = t * Ds;
            iDs = t * Da;
        }
        if (HESS) hess2(ra, rs, iDa, iDs);
        break;
    }
    case K_CUT: {
        // circular: k = 0, D_w = A_w^2; psi_s - psi_a = (C_s - C_a)/(psi_a + psi_s)
        const double R = fma(c[D_Q2], x2, y2);
        const double ta = c[D_CA] + R, ts = c[D_CS_] + R;
        const double ra = rsq64(ta), rs = rsq64(ts);
        const double pa = ta * ra, ps = ts * rs;
        const double A1 = pa + c[D_SA], A2 = ps + c[D_SS];
        const double sum = pa + ps;
        const double A12 = A1 * A2;
        const double R1 = rcp64(sum * A12);
        const double i12 = R1 * sum;
        if (GRAD) {
            const double g = c[D_DC] * (R1 * A12);
            const double t = (g + c[D_DS]) * i12;
            ax = t * xp;
            ay = t * yp;
        }
        if (HESS) {
            const double iA1 = i12 * A2, iA2 = i12 * A1;
            hess2(ra, rs, iA1 * iA1, iA2 * iA2);
        }
        break;
    }
    case K_ELL: {
        // lengths divided by k and quarter radius as in the two-core form
        const double ta = fma(c[D_EQ2], x2, fma(c[D_EK2I], y2, c[D_ECA]));
        const double ra = rsq2q(ta);
        const double A1 = fma(ta, ra, c[D_ESA]);
        const double B1 = fma(ta, ra, c[D_EQ2SA]);
        const double Da = fma(A1, A1, x2);
        double iDa = 0.0;
        if (GRAD) {
            const AtanRed ra_ = atan_reduce(xp, A1);
            const AtanhRed rh = atanh_reduce(yp, B1);
            const double den = ra_.den * rh.den;
            const double R2 = rcp64(HESS ? den * Da : den);
            const double RD = HESS ? R2 * Da : R2;
            const double b = ra_.num * (RD * rh.den);
            const double s = rh.num * (RD * ra_.den);
            if (HESS) iDa = R2 * den;
            ax = atan_finish(ra_, b, S);
            ay = atanh_finish(rh, s, S);
        } else if (HESS) {
            iDa = rcp64(Da);
        }
        if (HESS) hess1(ra, iDa);
        break;
    }
    default: {
        const double ta = c[D_CA] + fma(c[D_Q2], x2, y2);
        const double ra = rsq64(ta);
        const double iA1 = rcp64(ta * ra + c[D_SA]);
        if (GRAD) {
            ax = iA1 * xp;
            ay = iA1 * yp;
        }
        if (HESS) hess1(ra, iA1 * iA1);
        break;
    }
    }
    if (kind & K_SING) {
        // (an empty volatile statement keeps this a branch: the compiler may
        // not turn it into selects executed for every potential)
        asm volatile("");
        if ((dx == 0.0) & (dy == 0.0)) ax = ay = htr = hdf = hxy = 0.0;
    }
    // rotate back and accumulate, the prefactors folded into the rotation
    // constants (ax, ay, htr, hdf, hxy above carry no PF or HF)
    if (GRAD) {
        const double pfc = c[D_PFC], pfs = c[D_PFS];
        acc[0] = fma(pfc, ax, acc[0]);
        acc[0] = fma(-pfs, ay, acc[0]);
        acc[1] = fma(pfs, ax, acc[1]);
        acc[1] = fma(pfc, ay, acc[1]);
    }
    if (HESS) {
        // rotating by phi leaves the trace and turns (difference/2, psi_xy)
        // by 2 phi: acc[2] = T, acc[3] = U, acc[4] = V
        acc[2] = fma(c[D_HT], htr, acc[2]);
        acc[3] = fma(c[D_HCMH], hdf, acc[3]);
        acc[3] = fma(c[D_HCS2], hxy, acc[3]);
        acc[4] = fma(c[D_HCS], hdf, acc[4]);
        acc[4] = fma(-c[D_HCMS], hxy, acc[4]);
    }
}

// UNIF: every lane of the wave evaluates the same potential (the kind is read
// into a scalar register and its branches are uniform); otherwise each lane
// may hold a different potential and the branches diverge.
// SHORT: the two-core elliptical form first tries the shorter polynomials
// (worth it where most waves are far from every core, as on a map).
template <bool GRAD, bool HESS, bool SHORT = false>
__device__ __forceinline__ void eval_pot_f64_rel(const ConstD c, int kind, double dx, double dy,
                                                 double dyc, double dys, double acc[5],
                                                 const Series &S) {
    eval_pot_f64_impl<GRAD, HESS, SHORT>(c, kind, dx, dy, dyc, dys, acc, S);
}

// One point, the kind given (as on the uniform paths, read once per potential).
template <bool GRAD, bool HESS, bool SHORT = false>
__device__ __forceinline__ void eval_pot_f64_kind(const ConstD c, int kind, double x, double y,
                                                  double acc[5], const Series &S) {
    const double dy = y - c[D_Y0];
    eval_pot_f64_rel<GRAD, HESS, SHORT>(c, kind, x - c[D_X0], dy, dy * c[D_C], dy * c[D_S], acc,
                                        S);
}

template <bool GRAD, bool HESS, bool UNIF = true, bool SHORT = false>
__device__ __forceinline__ void eval_pot_f64(const ConstD c, double x, double y, double acc[5],
                                             const Series &S) {
    const int kind = UNIF ? uniform_kind(c[D_KIND]) : kind_bits(c[D_KIND]);
    eval_pot_f64_kind<GRAD, HESS, SHORT>(c, kind, x, y, acc, S);
}

// Deflection of one two-core elliptical potential (kind K_CUT | K_ELL, rcore >
// 0) at NP points per lane, added to acc[p][0..1], always through the
// full-range arctangent and hyperbolic arctangent reductions: no polynomial
// tier is tried first.  This suits points spread over the strong-lensing
// region, such as the constraint positions of the chi^2, where the ratios of
// nearly every wave leave the tiers' intervals (the tiers would be evaluated
// and thrown away, with their own reciprocal).  The NP evaluations are
// independent straight-line code that the compiler interleaves.  The steps
// and their rounding are those of the reduction path of eval_pot_f64 (the
// two cores' differences, one reciprocal for both reduced quotients).
//
// grad_cut_ell_point: one point's deflection in the potential's frame, before
// the prefactors and the rotation back (which grad_cut_ell_add applies); the
// constants may differ from lane to lane.
struct CutEllConsts {
    double x0, y0, cp, sp, eq2, ek2i, eca, dc, esa, ess, eq2sa, eq2ss;
};
__device__ __forceinline__ CutEllConsts cut_ell_consts(const ConstD c) {
    return CutEllConsts{c[D_X0],  c[D_Y0],  c[D_C],   c[D_S],   c[D_EQ2],   c[D_EK2I],
                        c[D_ECA], c[D_DC],  c[D_ESA], c[D_ESS], c[D_EQ2SA], c[D_EQ2SS]};
}
__device__ __forceinline__ void grad_cut_ell_point(const CutEllConsts &k, double x, double y,
                                                   double &ax, double &ay, const Series &S) {
    const double dx = x - k.x0, dy = y - k.y0;
    const double xp = fma(dx, k.cp, dy * k.sp);
    const double yp = fma(-k.sp, dx, dy * k.cp);
    const double x2 = xp * xp, y2 = yp * yp;
    const double ta = fma(k.eq2, x2, fma(k.ek2i, y2, k.eca));
    const double ts = ta + k.dc;
    const double ra = rsq2q(ta), rs = rsq2q(ts);
    const double A1 = fma(ta, ra, k.esa), A2 = fma(ts, rs, k.ess);
    const double B1 = fma(ta, ra, k.eq2sa), B2 = fma(ts, rs, k.eq2ss);
    const double Dx = fma(A1, A2, x2);
    const double Dy = fma(B1, B2, -y2);
    const double Nx = xp * (A2 - A1);
    const double Ny = yp * (B2 - B1);
    const AtanRed ra_ = atan_reduce(Nx, Dx);
    const AtanhRed rh = atanh_reduce(Ny, Dy);
    const double R3 = rcp64(ra_.den * rh.den);
    const double b = ra_.num * (R3 * rh.den);
    const double s = rh.num * (R3 * ra_.den);
    ax = atan_finish(ra_, b, S);
    ay = atanh_finish(rh, s, S);
}
// acc += the rotated, scaled deflection (pfc, pfs: the potential's D_PFC, D_PFS)
__device__ __forceinline__ void grad_cut_ell_add(double pfc, double pfs, double ax, double ay,
                                                 double *acc) {
    acc[0] = fma(pfc, ax, acc[0]);
    acc[0] = fma(-pfs, ay, acc[0]);
    acc[1] = fma(pfs, ax, acc[1]);
    acc[1] = fma(pfc, ay, acc[1]);
}
template <int NP, int W>
__device__ __forceinline__ void grad_cut_ell_full(const ConstD c, const double *x,
                                                  const double *y, double (*acc)[W],
                                                  const Series &S) {
    const CutEllConsts k = cut_ell_consts(c);
    const double pfc = c[D_PFC], pfs = c[D_PFS];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        double ax, ay;
        grad_cut_ell_point(k, x[p], y[p], ax, ay, S);
        grad_cut_ell_add(pfc, pfs, ax, ay, acc[p]);
    }
}

// ---------------------------------------------------------------------------
// FP32 building blocks: native reciprocal and reciprocal square root (about
// one unit in the last place), the same reductions, series to b^9/9
// (truncation below 1e-8 b).
__device__ __forceinline__ float frcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ float frsq(float v) { return __builtin_amdgcn_rsqf(v); }

struct AtanRedF {
    float num, den, base;
    bool big;
    float sign;
};
__device__ __forceinline__ AtanRedF atan_reduce_f(float N, float D) {
    const float u = fabsf(N);
    const bool big = u > D;
    const float lo = big ? D : u, hi = big ? u : D;
    const bool m1 = lo > 0.19891237f * hi, m2 = lo > 0.66817864f * hi;
    const float c = m2 ? 1.0f : (m1 ? 0.41421356f : 0.0f);
    AtanRedF r;
    r.num = fmaf(-c, hi, lo);
    r.den = fmaf(c, lo, hi);
    r.base = m2 ? 0.78539816f : (m1 ? 0.39269908f : 0.0f);
    r.big = big;
    r.sign = N;
    return r;
}
__device__ __forceinline__ float atan_poly_f(float b, const Series &S) {
    const float b2 = b * b;
    float p = S.atf[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) p = fmaf(p, b2, S.atf[i]);
    return fmaf(b * b2, p, b);
}
__device__ __forceinline__ float atan_finish_f(const AtanRedF &r, float b, const Series &S) {
    float t = atan_poly_f(b, S) + r.base;
    t = r.big ? 1.57079633f - t : t;
    return copysignf(t, r.sign);
}
struct AtanhRedF {
    float num, den;
    int k;
};
__device__ __forceinline__ AtanhRedF atanh_reduce_f(float N, float D) {
    const float P = D + N, Q = D - N;
    const float mp = __builtin_amdgcn_frexp_mantf(P), mq = __builtin_amdgcn_frexp_mantf(Q);
    int k = __builtin_amdgcn_frexp_expf(P) - __builtin_amdgcn_frexp_expf(Q);
    k += (mp > 1.41421356f * mq) ? 1 : 0;
    k -= (mq > 1.41421356f * mp) ? 1 : 0;
    const float Pk = __builtin_amdgcn_ldexpf(P, -k);
    AtanhRedF r;
    r.num = (k == 0) ? 2.0f * N : Pk - Q;
    r.den = Pk + Q;
    r.k = k;
    return r;
}
__device__ __forceinline__ float atanh_poly_f(float s, const Series &S) {
    const float s2 = s * s;
    float p = S.ahf[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) p = fmaf(p, s2, S.ahf[i]);
    return fmaf(s * s2, p, s);
}
// The same to the fifth power, for |b|, |s| within the first fifth of the
// intervals (the omitted terms are below 1e-9 relative there).
__device__ __forceinline__ float atan_poly_fs(float b, const Series &S) {
    const float b2 = b * b;
    return fmaf(b * b2, fmaf(S.atf[2], b2, S.atf[3]), b);
}
__device__ __forceinline__ float atanh_poly_fs(float s, const Series &S) {
    const float s2 = s * s;
    return fmaf(s * s2, fmaf(S.ahf[2], s2, S.ahf[3]), s);
}
__device__ __forceinline__ float atanh_finish_f(const AtanhRedF &r, float s, const Series &S) {
    return fmaf(0.34657359f, (float)r.k, atanh_poly_f(s, S));
}

// FP32 evaluation: offset and rotation in FP64 (|x| ~ 100" would lose
// ~1e-5" if formed in FP32), the rest in FP32.  out[] receives this
// potential's rotated contribution.
template <bool GRAD, bool HESS, bool SING, bool SHORT>
__device__ __forceinline__ void eval_pot_f32_impl(const ConstD c, const ConstF f, int kind,
                                                  double x, double y, float out[5],
                                                  const Series &S) {
    double dx = x - c[D_X0];
    double dy = y - c[D_Y0];
    bool zero = false;
    if (SING) {
        zero = (dx == 0.0) & (dy == 0.0);
        if (zero) dx = 1.0;
    }
    const double cpd = c[D_C], spd = c[D_S];
    const float xp = (float)fma(dx, cpd, dy * spd);
    const float yp = (float)fma(dy, cpd, -(dx * spd));
    const float x2 = xp * xp, y2 = yp * yp;
    // elliptical (K_ELL32): lengths divided by k, as in the FP64 form; psi_w^2
    // (the second core's as the first's plus C_s - C_a) and A_w, B_w by FMAs
    const float ta = fmaf(f[F_Q2], x2, fmaf(f[F_K2I], y2, f[F_CA]));
    float ax = 0.f, ay = 0.f, htr = 0.f, hdf = 0.f, hxy = 0.f;  // as in the FP64 form
    if (kind & K_CUT) {
        const float ts = ta + f[F_DC];
        const float ra = frsq(ta), rs = frsq(ts);
        const float pa = ta * ra, ps = ts * rs;
        const float A1 = fmaf(ta, ra, f[F_SA]), A2 = fmaf(ts, rs, f[F_SS]);
        float iDa = 0.f, iDs = 0.f;
        if (kind & K_ELL32) {
            // one reciprocal (quarter-rate) for the Hessian denominators and
            // one for the ratio denominators (their product would leave the
            // FP32 range)
            if (HESS) {
                const float Da = fmaf(A1, A1, x2), Ds = fmaf(A2, A2, x2);
                const float t = frcp(Da * Ds);
                iDa = t * Ds;
                iDs = t * Da;
            }
            if (GRAD) {
                const float B1 = fmaf(ta, ra, f[F_Q2SA]), B2 = fmaf(ts, rs, f[F_Q2SS]);
                const float Nx = xp * (A2 - A1);
                const float Dx = fmaf(A1, A2, x2);
                const float Ny = yp * (B2 - B1);
                const float Dy = fmaf(B1, B2, -y2);
                const float R2 = frcp(Dx * Dy);
                const float bf = Nx * (R2 * Dy), sf = Ny * (R2 * Dx);
                // (SHORT) a second, shorter tier as in the FP64 form
                if (SHORT) {
                    ax = atan_poly_fs(bf, S);
                    ay = atanh_poly_fs(sf, S);
                }
                if (!SHORT || !wave_all(fabsf(bf) <= (float)kAtanSMax,
                                        fabsf(sf) <= (float)kAtanhSMax)) {
                    if (wave_all(fabsf(bf) <= 0.19891237f, fabsf(sf) <= 0.17157287f)) {
                        ax = atan_poly_f(bf, S);
                        ay = atanh_poly_f(sf, S);
                    } else {
                        const AtanRedF ra_ = atan_reduce_f(Nx, Dx);
                        const AtanhRedF rh = atanh_reduce_f(Ny, Dy);
                        ax = atan_finish_f(ra_, ra_.num * frcp(ra_.den), S);
                        ay = atanh_finish_f(rh, rh.num * frcp(rh.den), S);
                    }
                }
            }
        } else {
            const float sum = pa + ps;
            const float A12 = A1 * A2;
            const float R1 = frcp(sum * A12);
            const float inv_sum = R1 * A12;
            const float i12 = R1 * sum;
            if (HESS) {
                const float iA1 = i12 * A2, iA2 = i12 * A1;
                iDa = iA1 * iA1;
                iDs = iA2 * iA2;
            }
            if (GRAD) {
                const float g = f[F_DC] * inv_sum;
                const float t = (g + f[F_DS]) * i12;
                ax = t * xp;
                ay = t * yp;
            }
        }
        if (HESS) {
            const float ha = ra * iDa, hs = rs * iDs;
            const float dh = ha - hs;
            htr = ra - rs;
            hdf = fmaf(y2 - x2, dh, fmaf(ha, f[F_EA], -(hs * f[F_ES])));
            hxy = (xp * yp) * dh;
        }
    } else {
        const float ra = frsq(ta);
        const float A1 = fmaf(ta, ra, f[F_SA]);
        const float B1 = fmaf(ta, ra, f[F_Q2SA]);
        float iDa = 0.f;
        if (kind & K_ELL32) {
            if (GRAD) {
                const AtanRedF ra_ = atan_reduce_f(xp, A1);
                const AtanhRedF rh = atanh_reduce_f(yp, B1);
                ax = atan_finish_f(ra_, ra_.num * frcp(ra_.den), S);
                ay = atanh_finish_f(rh, rh.num * frcp(rh.den), S);
            }
            if (HESS) iDa = frcp(fmaf(A1, A1, x2));
        } else {
            const float iA1 = frcp(A1);
            if (GRAD) {
                ax = iA1 * xp;
                ay = iA1 * yp;
            }
            iDa = iA1 * iA1;
        }
        if (HESS) {
            const float ha = ra * iDa;
            htr = ra;
            hdf = ha * ((y2 - x2) + f[F_EA]);
            hxy = (xp * yp) * ha;
        }
    }
    if (SING && zero) ax = ay = htr = hdf = hxy = 0.f;
    // rotate back, the prefactors folded into the rotation constants
    if (GRAD) {
        const float pfc = f[F_PFC], pfs = f[F_PFS];
        out[0] = fmaf(pfc, ax, -(pfs * ay));
        out[1] = fmaf(pfs, ax, pfc * ay);
    }
    if (HESS) {
        // out[2..4] = this potential's T, U, V
        out[2] = f[F_HT] * htr;
        out[3] = fmaf(f[F_HCMH], hdf, f[F_HCS2] * hxy);
        out[4] = fmaf(f[F_HCS], hdf, -(f[F_HCMS] * hxy));
    }
}

template <bool GRAD, bool HESS, bool SHORT = false>
__device__ __forceinline__ void eval_pot_f32_kind(const ConstD c, const ConstF f, int kind,
                                                  double x, double y, float out[5],
                                                  const Series &S) {
    if (kind & K_SING)
        eval_pot_f32_impl<GRAD, HESS, true, SHORT>(c, f, kind, x, y, out, S);
    else
        eval_pot_f32_impl<GRAD, HESS, false, SHORT>(c, f, kind, x, y, out, S);
}

template <bool GRAD, bool HESS, bool UNIF = true, bool SHORT = false>
__device__ __forceinline__ void eval_pot_f32(const ConstD c, const ConstF f, double x, double y,
                                             float out[5], const Series &S) {
    const int kind = UNIF ? uniform_kind(c[D_KIND]) : kind_bits(c[D_KIND]);
    eval_pot_f32_kind<GRAD, HESS, SHORT>(c, f, kind, x, y, out, S);
}

// Neumaier compensated addition: s + c carries the sum to about twice the
// working precision.
__device__ __forceinline__ void neumaier_add(float &s, float &c, float v) {
    const float t = s + v;
    c += (fabsf(s) >= fabsf(v)) ? ((s - t) + v) : ((v - t) + s);
    s = t;
}

// Second derivatives from the accumulated parts: psi_xx = T + U,
// psi_xy = V, psi_yy = T - U.
__device__ __forceinline__ void hess_of_parts(double T, double U, double V, double h[3]) {
    h[0] = T + U;
    h[1] = V;
    h[2] = T - U;
}

}  // namespace lens
