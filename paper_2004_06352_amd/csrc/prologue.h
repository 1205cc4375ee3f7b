// prologue.h -- derived constants of one potential (the parameter prologue).
// Shared by the table prologue kernels and the sampler's proposal kernel.
#pragma once

#include <math.h>

#include "eval.h"
#include "lens_internal.h"

namespace lens {

// Amplitude-form parameters of potential k -> its derived constants (FP64
// block and, with F32, its FP32 copy; entry k of tables with the given
// stride).  Invalid entries get NaN prefactors (their contribution is NaN) and
// raise ST_INVALID_TABLE.  LOG: the constant of the potential's logarithmic
// term (D_LC, read only by the lensing-potential kernel) is formed; without
// it that entry is NaN.
template <bool F32 = true, bool LOG = true>
__device__ __forceinline__ void prologue_values(double x0, double y0, double b0, double eps,
                                                double phi, double a, double s, int k,
                                                double *__restrict__ dd, float *__restrict__ df,
                                                int stride, int *status) {
    const bool cut = isfinite(s);
    const bool ok = isfinite(x0) && isfinite(y0) && isfinite(b0) && b0 >= 0.0 &&
                    isfinite(eps) && eps >= 0.0 && eps < 1.0 && isfinite(phi) &&
                    isfinite(a) && a >= 0.0 && !isnan(s) && s > a;
    // Below this ellipticity the elliptical closed forms agree with the
    // circular ones far below FP64 rounding (they differ at first order in
    // eps), while lengths divided by k would leave the FP64 range.
    const bool ell = eps > 1e-60;
    double c = 1.0, sn = 0.0;
    if (ell) {
        c = cos(phi);
        sn = sin(phi);
    }
    // One reciprocal of 1 + eps, one reciprocal square root of eps and one
    // reciprocal of s - a (estimates and a Newton step each) serve every
    // quotient below, instead of correctly rounded divisions (a few units in
    // the last place on the constants)
    const double ope = 1.0 + eps;
    const double r1 = rcp64(ope);
    const double hr = ell ? 0.5 * rsq64(eps) : 0.0;  // 1/(2 sqrt(eps))
    const double q = (1.0 - eps) * r1, q2 = q * q;
    const double Sa = (1.0 + eps) * a;
    const double Ss = cut ? (1.0 + eps) * s : 0.0;
    const double k1 = ell ? 4.0 * (eps * hr) * r1 : 0.0;  // 2 sqrt(eps)/(1 + eps)
    const double F = cut ? s * rcp64(s - a) : 1.0;
    const double om = 1.0 - eps;
    const double DC = cut ? om * om * ((s - a) * (s + a)) : 0.0;
    const double DS = cut ? (1.0 + eps) * (s - a) : 0.0;
    double PF = ell ? F * b0 * (1.0 - eps * eps) * hr : F * b0;
    double HF = F * b0 * om;
    const bool ell32 = eps > 1e-8;
    int kind = (ell ? K_ELL : 0) | (ell32 ? K_ELL32 : 0) | (cut ? K_CUT : 0) |
               (a == 0.0 ? K_SING : 0);
    if (!ok) {
        PF = NAN;
        HF = NAN;
        kind = K_INVALID | K_CUT | K_ELL | K_ELL32;
        atomicOr(status, ST_INVALID_TABLE);
    }
    double v[NDER];
    v[D_X0] = x0;
    v[D_Y0] = y0;
    v[D_C] = c;
    v[D_S] = sn;
    v[D_PFC] = PF * c;
    v[D_PFS] = PF * sn;
    // Hessian constants: the FP64 evaluation of an elliptical potential
    // leaves a factor k on the trace and 1/k^3 on the other parts, and works
    // with quarter radii (its 1/psi_w carry a factor 4, taken out here by h4)
    const double kap = ell ? ope * hr : 1.0, kap2 = kap * kap, kap3 = kap2 * kap;  // 1/k
    const double h4 = ell ? 0.25 : 1.0;
    const double hcms = HF * (c * c - sn * sn), hcs = HF * (c * sn);
    v[D_HT] = h4 * (kap * (0.5 * HF));
    v[D_HCMS] = h4 * (kap3 * hcms);
    v[D_HCMH] = h4 * (kap3 * (0.5 * hcms));
    v[D_HCS] = h4 * (kap3 * hcs);
    v[D_HCS2] = h4 * (kap3 * (2.0 * hcs));
    v[D_Q2] = q2;
    v[D_CA] = q2 * Sa * Sa;
    v[D_CS_] = q2 * Ss * Ss;
    v[D_SA] = Sa;
    v[D_SS] = Ss;
    v[D_Q2SA] = q2 * Sa;
    v[D_Q2SS] = q2 * Ss;
    v[D_DC] = h4 * (kap2 * DC);
    v[D_DS] = DS;
    const double pk = ell ? PF * k1 : 0.0;  // F b0 (1 - eps)
    v[D_LA] = 0.5 * pk * Sa;
    v[D_LS] = 0.5 * pk * Ss;
    v[D_LC] = !LOG ? NAN : (ell ? pk * log(k1) * (Sa - Ss) : 0.0);
    v[D_PF] = PF;
    v[D_EA] = Sa * (q2 * Sa - Sa);
    v[D_ES] = Ss * (q2 * Ss - Ss);
    v[D_EQ2] = h4 * (kap2 * q2);
    v[D_EK2I] = h4 * kap2;
    v[D_ECA] = h4 * (kap2 * v[D_CA]);
    v[D_ECS] = h4 * (kap2 * v[D_CS_]);
    v[D_ESA] = kap * Sa;
    v[D_ESS] = kap * Ss;
    v[D_EQ2SA] = kap * v[D_Q2SA];
    v[D_EQ2SS] = kap * v[D_Q2SS];
    v[D_KIND] = __longlong_as_double((long long)kind);  // bit pattern, low word = kind
    for (int i = 0; i < NDER; ++i) dd[(size_t)i * stride + k] = v[i];
    if (!F32) return;
    // the FP32 evaluation's own scaling (see the FP32 table's layout)
    const double g = ell32 ? kap : 1.0, g2 = g * g, g3 = g2 * g;
    const double PF32 = ell32 ? PF : (ok ? F * b0 : NAN);
    const double fv[NDERF] = {g * (0.5 * HF), g3 * (0.5 * hcms), g3 * hcs, g3 * (2.0 * hcs),
                              g3 * hcms,      g2 * q2,           g2 * v[D_CA], g2 * v[D_CS_],
                              g * Sa,         g * Ss,            g * v[D_Q2SA], g * v[D_Q2SS],
                              g2,             g2 * DC,           DS,        PF32 * c,
                              PF32 * sn,      v[D_EA],           v[D_ES]};
    for (int i = 0; i < NDERF; ++i) df[(size_t)i * stride + k] = (float)fv[i];
}

}  // namespace lens
