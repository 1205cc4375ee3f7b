// prologue.h -- derived constants of one potential (the parameter prologue).
// Shared by the table prologue kernels and the sampler's proposal kernel.
#pragma once

#include <math.h>

#include "lens_internal.h"

namespace lens {

// Amplitude-form parameters of potential k -> its derived constants (FP64
// block and, with F32, its FP32 copy; entry k of tables with the given
// stride).  Invalid entries get NaN prefactors (their contribution is NaN) and
// raise ST_INVALID_TABLE.
template <bool F32 = true>
__device__ __forceinline__ void prologue_values(double x0, double y0, double b0, double eps,
                                                double phi, double a, double s, int k,
                                                double *__restrict__ dd, float *__restrict__ df,
                                                int stride, int *status) {
    const bool cut = isfinite(s);
    const bool ok = isfinite(x0) && isfinite(y0) && isfinite(b0) && b0 >= 0.0 &&
                    isfinite(eps) && eps >= 0.0 && eps < 1.0 && isfinite(phi) &&
                    isfinite(a) && a >= 0.0 && !isnan(s) && s > a;
    const bool ell = eps > 0.0;
    double c = 1.0, sn = 0.0;
    if (ell) {
        c = cos(phi);
        sn = sin(phi);
    }
    const double q = (1.0 - eps) / (1.0 + eps), q2 = q * q;
    const double Sa = (1.0 + eps) * a;
    const double Ss = cut ? (1.0 + eps) * s : 0.0;
    const double k1 = ell ? 2.0 * sqrt(eps) / (1.0 + eps) : 0.0;
    const double F = cut ? s / (s - a) : 1.0;
    const double om = 1.0 - eps;
    const double DC = cut ? om * om * ((s - a) * (s + a)) : 0.0;
    const double DS = cut ? (1.0 + eps) * (s - a) : 0.0;
    double PF = ell ? F * b0 * (1.0 - eps * eps) / (2.0 * sqrt(eps)) : F * b0;
    double HF = F * b0 * om;
    int kind = (ell ? K_ELL : 0) | (cut ? K_CUT : 0) | (a == 0.0 ? K_SING : 0);
    if (!ok) {
        PF = NAN;
        HF = NAN;
        kind = K_INVALID | K_CUT | K_ELL;
        atomicOr(status, ST_INVALID_TABLE);
    }
    double v[NDER];
    v[D_X0] = x0;
    v[D_Y0] = y0;
    v[D_C] = c;
    v[D_S] = sn;
    v[D_PFC] = PF * c;
    v[D_PFS] = PF * sn;
    v[D_HT] = 0.5 * HF;
    v[D_HCMS] = HF * (c * c - sn * sn);
    v[D_HCMH] = 0.5 * v[D_HCMS];
    v[D_HCS] = HF * (c * sn);
    v[D_HCS2] = 2.0 * v[D_HCS];
    v[D_Q2] = q2;
    v[D_CA] = q2 * Sa * Sa;
    v[D_CS_] = q2 * Ss * Ss;
    v[D_SA] = Sa;
    v[D_SS] = Ss;
    v[D_Q2SA] = q2 * Sa;
    v[D_Q2SS] = q2 * Ss;
    v[D_K] = k1;
    v[D_K2] = k1 * k1;
    v[D_DC] = DC;
    v[D_DS] = DS;
    v[D_Q2DS] = q2 * DS;
    v[D_PF] = PF;
    v[D_EA] = Sa * (q2 * Sa - Sa);
    v[D_ES] = Ss * (q2 * Ss - Ss);
    v[D_KIND] = __longlong_as_double((long long)kind);  // bit pattern, low word = kind
    for (int i = 0; i < NDER; ++i) dd[(size_t)i * stride + k] = v[i];
    if (!F32) return;
    const double fv[NDERF] = {v[D_HT],   v[D_HCMH],  v[D_HCS],    v[D_HCS2], v[D_HCMS],
                              q2,        v[D_CA],    v[D_CS_],    Sa,        Ss,
                              v[D_Q2SA], v[D_Q2SS],  k1,          v[D_K2],   DC,
                              DS,        v[D_Q2DS],  v[D_PFC],    v[D_PFS],  v[D_EA],
                              v[D_ES]};
    for (int i = 0; i < NDERF; ++i) df[(size_t)i * stride + k] = (float)fv[i];
}

}  // namespace lens
