// eval.h -- per-potential deflection / second-derivative evaluation on gfx950.
//
// One call evaluates one potential at one point and adds its contribution to
// the accumulators.  Every lane of a wave evaluates the same potential at the
// same time, so the branches on the potential's kind are uniform across the
// wave (the kind is read into a scalar register).
//
// Math (Keeton 2001 closed forms of the cored isothermal ellipsoid, mapped to
// the Kassiola-Kovner ellipticity of the dPIE; the paper's Sec. 2.2 model
// parameters, summed per Sec. 4.1 Eq. (10) and Sec. 2.4 Eqs. (7)-(9)):
//   two cores a < s combine as F (P_a - P_s); the arctangent and hyperbolic
//   arctangent differences use
//     atan(kx/A_a) - atan(kx/A_s)   = atan2(k x (A_s - A_a), A_a A_s + k^2 x^2)
//     atanh(ky/B_a) - atanh(ky/B_s) = atanh(k y (B_s - B_a) / (B_a B_s - k^2 y^2))
//   (both arguments have the same sign, so no branch correction is needed),
//   and atanh(z) = log1p(2z/(1-z))/2.  A_s - A_a = (C_s-C_a)/(psi_a+psi_s) + (S_s-S_a).
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

__device__ __forceinline__ int uniform_kind(double k) {
    return __builtin_amdgcn_readfirstlane((int)k);
}

template <bool GRAD, bool HESS>
__device__ __forceinline__ void eval_pot_f64(const ConstD c, double x, double y, double acc[5]) {
    const int kind = uniform_kind(c[D_KIND]);
    double dx = x - c[D_X0];
    double dy = y - c[D_Y0];
    bool zero = false;
    if (kind & K_SING) {
        zero = (dx == 0.0) & (dy == 0.0);
        if (zero) dx = 1.0;  // any regular point; the contribution is dropped
    }
    const double cp = c[D_C], sp = c[D_S];
    const double xp = dx * cp + dy * sp;
    const double yp = dy * cp - dx * sp;
    const double x2 = xp * xp, y2 = yp * yp;
    const double R = c[D_Q2] * x2 + y2;
    double ax = 0.0, ay = 0.0, hxx = 0.0, hxy = 0.0, hyy = 0.0;
    if (kind & K_CUT) {
        const double pa = sqrt(c[D_CA] + R);
        const double ps = sqrt(c[D_CS_] + R);
        const double A1 = pa + c[D_SA], A2 = ps + c[D_SS];
        if (GRAD) {
            const double g = c[D_DC] / (pa + ps);
            if (kind & K_ELL) {
                const double B1 = pa + c[D_Q2SA], B2 = ps + c[D_Q2SS];
                const double k = c[D_K], k2 = c[D_K2];
                const double Nx = k * xp * (g + c[D_DS]);
                const double Dx = A1 * A2 + k2 * x2;
                const double Ny = k * yp * (g + c[D_Q2DS]);
                const double Dy = B1 * B2 - k2 * y2;
                ax = c[D_PF] * atan2(Nx, Dx);
                ay = 0.5 * c[D_PF] * log1p(2.0 * Ny / (Dy - Ny));
            } else {
                const double t = c[D_PF] * (g + c[D_DS]) / (A1 * A2);
                ax = t * xp;
                ay = t * yp;
            }
        }
        if (HESS) {
            const double k2x2 = c[D_K2] * x2;
            const double Da = A1 * A1 + k2x2, Ds = A2 * A2 + k2x2;
            const double ha = c[D_HF] / (pa * Da), hs = c[D_HF] / (ps * Ds);
            hxx = ha * (c[D_CA] + y2 + c[D_SA] * pa) - hs * (c[D_CS_] + y2 + c[D_SS] * ps);
            hyy = ha * (c[D_SA2] + x2 + c[D_SA] * pa) - hs * (c[D_SS2] + x2 + c[D_SS] * ps);
            hxy = -xp * yp * (ha - hs);
        }
    } else {
        const double pa = sqrt(c[D_CA] + R);
        const double A1 = pa + c[D_SA];
        if (GRAD) {
            if (kind & K_ELL) {
                const double k = c[D_K];
                const double B1 = pa + c[D_Q2SA];
                const double ky = k * yp;
                ax = c[D_PF] * atan2(k * xp, A1);
                ay = 0.5 * c[D_PF] * log1p(2.0 * ky / (B1 - ky));
            } else {
                const double t = c[D_PF] / A1;
                ax = t * xp;
                ay = t * yp;
            }
        }
        if (HESS) {
            const double Da = A1 * A1 + c[D_K2] * x2;
            const double ha = c[D_HF] / (pa * Da);
            hxx = ha * (c[D_CA] + y2 + c[D_SA] * pa);
            hyy = ha * (c[D_SA2] + x2 + c[D_SA] * pa);
            hxy = -xp * yp * ha;
        }
    }
    if (zero) ax = ay = hxx = hxy = hyy = 0.0;
    if (GRAD) {
        acc[0] += cp * ax - sp * ay;
        acc[1] += sp * ax + cp * ay;
    }
    if (HESS) {
        const double c2 = c[D_C2], s2 = c[D_S2], cs = c[D_CS], cms = c[D_CMS];
        const double t = 2.0 * cs * hxy;
        acc[2] += c2 * hxx - t + s2 * hyy;
        acc[3] += cs * (hxx - hyy) + cms * hxy;
        acc[4] += s2 * hxx + t + c2 * hyy;
    }
}

__device__ __forceinline__ float frcp(float v) { return __builtin_amdgcn_rcpf(v); }

// FP32 evaluation: offset and rotation in FP64 (|x| ~ 100" would lose
// ~1e-5" if formed in FP32), the rest in FP32.  out[] receives this
// potential's rotated contribution.
template <bool GRAD, bool HESS>
__device__ __forceinline__ void eval_pot_f32(const ConstD c, const ConstF f, double x, double y,
                                             float out[5]) {
    const int kind = uniform_kind(c[D_KIND]);
    double dx = x - c[D_X0];
    double dy = y - c[D_Y0];
    bool zero = false;
    if (kind & K_SING) {
        zero = (dx == 0.0) & (dy == 0.0);
        if (zero) dx = 1.0;
    }
    const double cpd = c[D_C], spd = c[D_S];
    const float xp = (float)(dx * cpd + dy * spd);
    const float yp = (float)(dy * cpd - dx * spd);
    const float x2 = xp * xp, y2 = yp * yp;
    const float R = f[F_Q2] * x2 + y2;
    float ax = 0.f, ay = 0.f, hxx = 0.f, hxy = 0.f, hyy = 0.f;
    if (kind & K_CUT) {
        const float pa = __builtin_sqrtf(f[F_CA] + R);
        const float ps = __builtin_sqrtf(f[F_CS_] + R);
        const float A1 = pa + f[F_SA], A2 = ps + f[F_SS];
        if (GRAD) {
            const float g = f[F_DC] * frcp(pa + ps);
            if (kind & K_ELL) {
                const float B1 = pa + f[F_Q2SA], B2 = ps + f[F_Q2SS];
                const float k = f[F_K], k2 = f[F_K2];
                const float Nx = k * xp * (g + f[F_DS]);
                const float Dx = A1 * A2 + k2 * x2;
                const float Ny = k * yp * (g + f[F_Q2DS]);
                const float Dy = B1 * B2 - k2 * y2;
                ax = f[F_PF] * atan2f(Nx, Dx);
                ay = 0.5f * f[F_PF] * log1pf(2.0f * Ny * frcp(Dy - Ny));
            } else {
                const float t = f[F_PF] * (g + f[F_DS]) * frcp(A1 * A2);
                ax = t * xp;
                ay = t * yp;
            }
        }
        if (HESS) {
            const float k2x2 = f[F_K2] * x2;
            const float Da = A1 * A1 + k2x2, Ds = A2 * A2 + k2x2;
            const float ha = f[F_HF] * frcp(pa * Da), hs = f[F_HF] * frcp(ps * Ds);
            hxx = ha * (f[F_CA] + y2 + f[F_SA] * pa) - hs * (f[F_CS_] + y2 + f[F_SS] * ps);
            hyy = ha * (f[F_SA2] + x2 + f[F_SA] * pa) - hs * (f[F_SS2] + x2 + f[F_SS] * ps);
            hxy = -xp * yp * (ha - hs);
        }
    } else {
        const float pa = __builtin_sqrtf(f[F_CA] + R);
        const float A1 = pa + f[F_SA];
        if (GRAD) {
            if (kind & K_ELL) {
                const float k = f[F_K];
                const float B1 = pa + f[F_Q2SA];
                const float ky = k * yp;
                ax = f[F_PF] * atan2f(k * xp, A1);
                ay = 0.5f * f[F_PF] * log1pf(2.0f * ky * frcp(B1 - ky));
            } else {
                const float t = f[F_PF] * frcp(A1);
                ax = t * xp;
                ay = t * yp;
            }
        }
        if (HESS) {
            const float Da = A1 * A1 + f[F_K2] * x2;
            const float ha = f[F_HF] * frcp(pa * Da);
            hxx = ha * (f[F_CA] + y2 + f[F_SA] * pa);
            hyy = ha * (f[F_SA2] + x2 + f[F_SA] * pa);
            hxy = -xp * yp * ha;
        }
    }
    if (zero) ax = ay = hxx = hxy = hyy = 0.f;
    if (GRAD) {
        const float cp = (float)cpd, sp = (float)spd;
        out[0] = cp * ax - sp * ay;
        out[1] = sp * ax + cp * ay;
    }
    if (HESS) {
        const float c2 = f[F_C2], s2 = f[F_S2], cs = f[F_CS], cms = f[F_CMS];
        const float t = 2.0f * cs * hxy;
        out[2] = c2 * hxx - t + s2 * hyy;
        out[3] = cs * (hxx - hyy) + cms * hxy;
        out[4] = s2 * hxx + t + c2 * hyy;
    }
}

// Neumaier compensated addition: s + c carries the sum to about twice the
// working precision.
__device__ __forceinline__ void neumaier_add(float &s, float &c, float v) {
    const float t = s + v;
    c += (fabsf(s) >= fabsf(v)) ? ((s - t) + v) : ((v - t) + s);
    s = t;
}

}  // namespace lens
