// lens_internal.h -- layouts and launch wrappers shared by the library's
// translation units (device side and host side).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lenshpc.h"
#include "series_coeffs.h"

namespace lens {

// ---------------------------------------------------------------------------
// Derived per-potential constants (output of the parameter prologue).
//
// Each potential is a dPIE = F (P_a - P_s): two cored isothermal ellipsoids
// with cores w = a (rcore) and w = s (rcut), F = s/(s-a).  In the frame of
// the potential, with q = (1-eps)/(1+eps), k = sqrt(1-q^2) = 2 sqrt(eps)/(1+eps),
// S_w = (1+eps) w and R = q^2 x'^2 + y'^2, each core has
//   psi_w = sqrt(q^2 S_w^2 + R),  A_w = psi_w + S_w,  B_w = psi_w + q^2 S_w,
// deflection  P b0' [atan(k x'/A_w), atanh(k y'/B_w)] (P = (1-eps^2)/(2 sqrt eps))
// and Hessian b0 (1-eps)/(psi_w D_w) [C_w + y'^2 + S_w psi_w, -x'y',
// S_w^2 + x'^2 + S_w psi_w], D_w = A_w^2 + k^2 x'^2.
// The GPU path subtracts the two cores' arctangents and hyperbolic arctangents
// in closed form (one atan2 and one log1p per potential instead of two of
// each).  For eps > 0 it works with every length divided by k (psi_w/k, A_w/k,
// B_w/k; the D_E* entries), so that the ratios lose their k and D_w/k^2 =
// (A_w/k)^2 + x'^2; the numerators x'(A_s - A_a) and y'(B_s - B_a) are formed
// directly (their rounding is a few units of the cores' own terms).  Since
// q^2 + k^2 = 1 and C_w = S_w q^2 S_w, the trace of a core's bracket is D_w: a
// core's psi_xx + psi_yy is b0 (1-eps)/psi_w and needs no quotient, and
// psi_xx - psi_yy is (y'^2 - x'^2 + E_w)/(psi_w D_w), E_w = S_w (q^2 S_w - S_w).
// The second derivatives are accumulated as a trace part T, a difference part
// U and the off-diagonal V in the frame of the sum: psi_xx = T + U,
// psi_yy = T - U, psi_xy = V.
// ---------------------------------------------------------------------------
enum DerivedIndex : int {
    D_X0 = 0, D_Y0, D_C, D_S,          // centre, cos(phi), sin(phi)
    D_PFC, D_PFS,                      // PF c, PF s: deflection rotated back
    D_HT, D_HCMH, D_HCS, D_HCS2, D_HCMS,  // HF/2, HF (c^2 - s^2)/2, HF c s, 2 HF c s, HF (c^2 - s^2);
                                       // for eps > 0 times 1/k (D_HT) and 1/k^3 (the rest),
                                       // and 1/4 (the quarter radii below)
    D_Q2,                              // q^2
    D_CA, D_CS_, D_SA, D_SS,           // C_a = q^2 S_a^2, C_s, S_a, S_s
    D_Q2SA, D_Q2SS,                    // q^2 S_a, q^2 S_s
    D_DC, D_DS,                        // C_s - C_a (divided by 4 k^2 for eps > 0, as the
                                       // D_EQ2 .. D_ECS entries), S_s - S_a
    D_LA, D_LS, D_LC,                  // eps > 0, the potential's log terms: PF k S_a/2,
                                       // PF k S_s/2, PF k ln(k) (S_a - S_s)
    D_PF,                              // deflection prefactor (F included)
    D_EA, D_ES,                        // E_a, E_s
    // eps > 0: the lengths of the closed form divided by k, the squared ones
    // also by 4 (a quarter of the squared radius R/k^2; unscaled for eps = 0)
    D_EQ2, D_EK2I,                     // q^2/(4 k^2), 1/(4 k^2)
    D_ECA, D_ECS, D_ESA, D_ESS,        // C_a/(4 k^2), C_s/(4 k^2), S_a/k, S_s/k
    D_EQ2SA, D_EQ2SS,                  // q^2 S_a/k, q^2 S_s/k
    D_KIND,                            // kind bits: low word of the entry's bit pattern
    NDER
};
// Float copy of the constants used after the FP64 offset/rotation step.  For
// eps > 1e-8 (K_ELL32) the FP32 evaluation takes the lengths divided by k as
// the FP64 one does (F_Q2 .. F_Q2SS, F_K2I and the Hessian constants as the
// D_E* and D_H* entries without their factor 1/4); below, it takes the
// circular forms (they differ from
// the elliptical ones at first order in eps, far below FP32 rounding), with
// the circular prefactor in F_PFC, F_PFS.
enum DerivedIndexF : int {
    F_HT = 0, F_HCMH, F_HCS, F_HCS2, F_HCMS,
    F_Q2, F_CA, F_CS_, F_SA, F_SS, F_Q2SA, F_Q2SS, F_K2I,
    F_DC, F_DS,                        // C_s - C_a (in the FP32 length units), S_s - S_a
    F_PFC, F_PFS,                      // PF c, PF s
    F_EA, F_ES,
    NDERF
};

enum KindBits : int {
    K_ELL = 1,      // eps > 0: elliptical closed forms
    K_CUT = 2,      // rcut finite: two cores
    K_SING = 4,     // rcore == 0: singular centre (zero contribution there)
    K_INVALID = 8,  // bad parameters: contributes NaN
    K_ELL32 = 16,   // eps > 1e-8: elliptical closed forms in the FP32 evaluation
};

// Derived table in device memory: double block [NDER][stride], then float
// block [NDERF][stride].
struct Derived {
    const double *d;
    const float *f;
    int n;
    int stride;
};

inline size_t derived_bytes(int n) {
    size_t stride = ((size_t)n + 63) / 64 * 64;
    if (stride == 0) stride = 64;
    return stride * (NDER * sizeof(double) + NDERF * sizeof(float));
}
inline int derived_stride(int n) {
    int s = (n + 63) / 64 * 64;
    return s == 0 ? 64 : s;
}

// Grid point coordinate o + i*d with the product and the sum rounded
// separately (no fused multiply-add), as the grid definition states.
__device__ __forceinline__ double grid_coord(double o, int i, double d) {
#pragma clang fp contract(off)
    return o + (double)i * d;
}

struct PotSoA {
    const double *x0, *y0, *b0, *eps, *phi, *rcore, *rcut;
};

// Polynomial coefficients of atan and atanh (Horner order, highest first):
// FP64 Chebyshev interpolants on the reduced intervals (series_coeffs.h),
// FP32 Taylor coefficients.  They travel as a kernel argument so that the
// kernels read them from scalar registers (literal FP64 constants would be
// held in vector registers and copied before every fused multiply-add).
struct Series {
    double at[LENS_ATAN_N];   // atan(b) = b + b^3 p(b^2), p ~ -1/3 + b^2/5 - ...
    double ah[LENS_ATANH_N];  // atanh(s) = s + s^3 q(s^2), q ~ 1/3 + s^2/5 + ...
    double ats[LENS_ATAN_S_N];    // the same pair on the first fifth of each interval
    double ahs[LENS_ATANH_S_N];
    float atf[4];             // 1/9, -1/7, 1/5, -1/3
    float ahf[4];             // 1/9, 1/7, 1/5, 1/3
};
inline Series make_series() {
    Series S;
    const double at[LENS_ATAN_N] = {LENS_ATAN_COEFFS};
    const double ah[LENS_ATANH_N] = {LENS_ATANH_COEFFS};
    for (int i = 0; i < LENS_ATAN_N; ++i) S.at[i] = at[i];
    for (int i = 0; i < LENS_ATANH_N; ++i) S.ah[i] = ah[i];
    const double ats[LENS_ATAN_S_N] = {LENS_ATAN_S_COEFFS};
    const double ahs[LENS_ATANH_S_N] = {LENS_ATANH_S_COEFFS};
    for (int i = 0; i < LENS_ATAN_S_N; ++i) S.ats[i] = ats[i];
    for (int i = 0; i < LENS_ATANH_S_N; ++i) S.ahs[i] = ahs[i];
    for (int i = 0; i < 4; ++i) S.atf[i] = (float)(((i % 2) ? -1.0 : 1.0) / (9 - 2 * i));
    for (int i = 0; i < 4; ++i) S.ahf[i] = (float)(1.0 / (9 - 2 * i));
    return S;
}

struct GridArgs {
    int nx, ny;
    double x0, y0, dx, dy;
};


// status word bits written by device code
enum StatusBits : int {
    ST_INVALID_TABLE = 1,
    ST_OVERFLOW = 2,
    ST_DOMAIN = 4,   // an exact orientation test met a coordinate outside its exact domain
    ST_BAD_F = 8,    // a source's Dls/Ds outside (0, 1]
};

// ---------------------------------------------------------------------------
// Launch wrappers (defined in the .hip translation units).  Each returns the
// HIP error of the launch.
// ---------------------------------------------------------------------------
hipError_t launch_zero_i32(int *p, int n, hipStream_t st);
// Parts of a derived table a prologue writes besides the FP64 block: the
// FP32 copy (PRO_F32, for the FP32-evaluation precisions) and the constant of
// the logarithmic term (PRO_LOG, for the lensing-potential kernel).
enum PrologueParts : int { PRO_F32 = 1, PRO_LOG = 2 };
hipError_t launch_prologue2(PotSoA a, int na, double *dda, float *dfa, int sa, PotSoA b, int nb,
                            double *ddb, float *dfb, int sb, int *status, int parts,
                            hipStream_t st);
hipError_t launch_prologue(PotSoA in, int n, double *dd, float *df, int stride, int *status,
                           int parts, hipStream_t st);
hipError_t launch_phys_to_amp(const double *sigma, const double *e, int n, int convention,
                              double *b0, double *eps, int *status, hipStream_t st);

struct MapLaunch {
    Derived tab;
    GridArgs grid;
    double dlsds;
    void *out[5];  // ax, ay, hxx, hxy, hyy (NULL = not stored)
    void *dout[6] = {};     // derived: kappa, gamma1, gamma2, gamma, mu, det
    bool derived = false;   // store the derived maps of the second derivatives instead of out[]
    int prec;
    bool grad, hess;
    lens_map_tuning_t tune;
};
hipError_t launch_map(const MapLaunch &m, hipStream_t st);
bool map_tuning_valid(const lens_map_tuning_t &t);

}  // namespace lens
