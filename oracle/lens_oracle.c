/*
 * lens_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU reference for the lens-gradient
 * hot path of Lenstool-HPC (Schaefer, Fourestey & Kneib, arXiv:2004.06352).
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may call it.  It shares no code, header, table or helper with the
 * GPU library; every loop runs in the order the method states it, with no
 * blocking, fusion or reordering.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 * (FMA contraction off: every product and sum below is rounded on its own).
 *
 * What is computed, and where it comes from:
 *   - Lens equation beta = theta - alpha(theta), alpha = grad psi: paper Sec. 2.1, Eq. (1).
 *   - Deflection map = sum over potentials of each potential's gradient: Sec. 4.1, Eq. (10).
 *   - Hessian (second derivatives) map, the input of kappa/gamma/mu: Sec. 2.4, Eqs. (7)-(9);
 *     the derived maps themselves (kappa, shear, det A^-1, mu): Sec. 2.4 with
 *     Sec. 2.1's magnification matrix.
 *   - The paper names only the parameters of its sub-halo models (centre,
 *     velocity dispersion, ellipticity, orientation, profile parameters;
 *     Sec. 2.2) and cites Eliasdottir et al. (2007) for them.  The profile
 *     used is that paper's dPIE: a difference of two cored isothermal
 *     ellipsoids (core radius a, cut radius s), with the Kassiola & Kovner
 *     (1993) elliptical form.  The closed forms of each cored ellipsoid are
 *     those of Keeton (2001, "A catalog of mass models"), softened isothermal
 *     ellipsoid, under the mapping b = b0(1+eps), q = (1-eps)/(1+eps),
 *     s_K = (1+eps) w.
 *   - Source-plane chi^2: unlens every image, take the barycentre of the
 *     unlensed positions per system (Sec. 2.2, Fig. 3) and sum the squared
 *     scatter over sigma^2 (Eq. (6) evaluated in the source plane).
 *   - Image-plane chi^2 by brute-force grid inversion: unlens a triangulated
 *     image-plane grid, find every triangle whose source-plane image contains
 *     the source, assign found images to the closest constraint and sum
 *     Eq. (6) (Sec. 2.3, Fig. 4; Sec. 4.2, Fig. 7).
 *
 * Channel order of every 5-vector below: [alpha_x, alpha_y, psi_xx, psi_xy, psi_yy].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* One cored isothermal ellipsoid, in the frame aligned with its major axis.  */
/* ------------------------------------------------------------------------- */
/* Deflection and Hessian of the cored isothermal ellipsoid with convergence
 *   kappa_w(x', y') = (b0/2) / sqrt(w^2 + x'^2/(1+eps)^2 + y'^2/(1-eps)^2)
 * (Kassiola & Kovner 1993 ellipticity eps; Keeton 2001 closed forms). */
static void cie_core(double b0, double eps, double w, double xp, double yp,
                     double out[5])
{
    double q = (1.0 - eps) / (1.0 + eps);
    double q2 = q * q;
    double S = (1.0 + eps) * w;
    double psi = sqrt(q2 * (S * S + xp * xp) + yp * yp);
    double ax, ay;
    if (eps > 0.0) {
        /* k = sqrt(1 - q^2), written so that it does not cancel */
        double k = 2.0 * sqrt(eps) / (1.0 + eps);
        double pref = b0 * (1.0 - eps * eps) / (2.0 * sqrt(eps));
        ax = pref * atan(k * xp / (psi + S));
        ay = pref * atanh(k * yp / (psi + q2 * S));
    } else {
        ax = b0 * xp / (psi + w);
        ay = b0 * yp / (psi + w);
    }
    double D = (1.0 + q2) * S * S + 2.0 * psi * S + xp * xp + yp * yp;
    double h = b0 * (1.0 - eps) / psi;
    out[0] = ax;
    out[1] = ay;
    out[2] = h * (q2 * S * S + yp * yp + S * psi) / D;  /* xx */
    out[3] = -h * xp * yp / D;                         /* xy */
    out[4] = h * (S * S + xp * xp + S * psi) / D;      /* yy */
}

/* Rotate a frame-aligned 5-vector back to sky axes (position angle phi,
 * counter-clockwise from +x).  alpha -> R alpha, H -> R H R^T. */
static void rotate_back(double c, double s, const double v[5], double o[5])
{
    o[0] = c * v[0] - s * v[1];
    o[1] = s * v[0] + c * v[1];
    o[2] = c * c * v[2] - 2.0 * c * s * v[3] + s * s * v[4];
    o[3] = c * s * (v[2] - v[4]) + (c * c - s * s) * v[3];
    o[4] = s * s * v[2] + 2.0 * c * s * v[3] + c * c * v[4];
}

/* The same rotation applied to magnitudes: a bound on the size of the terms
 * each rotated channel is summed from.  Used as the condition scale of the
 * comparison tolerance, never in the result. */
static void rotate_back_abs(double c, double s, const double v[5], double o[5])
{
    double ac = fabs(c), as = fabs(s);
    o[0] = ac * fabs(v[0]) + as * fabs(v[1]);
    o[1] = as * fabs(v[0]) + ac * fabs(v[1]);
    o[2] = c * c * fabs(v[2]) + 2.0 * ac * as * fabs(v[3]) + s * s * fabs(v[4]);
    o[3] = ac * as * (fabs(v[2]) + fabs(v[4])) + fabs(c * c - s * s) * fabs(v[3]);
    o[4] = s * s * fabs(v[2]) + 2.0 * ac * as * fabs(v[3]) + c * c * fabs(v[4]);
}

/* One dPIE potential p = {x0, y0, b0, eps, phi, rcore, rcut} at sky point
 * (x, y), at Dls/Ds = 1.  dPIE = F (P_a - P_s), F = s/(s-a); rcut = +inf
 * drops the cut term (F = 1).  A potential with rcore = 0 contributes zero
 * exactly at its own centre (the only singular point).  mag (may be NULL)
 * receives F (|R P_a| + |R P_s|) per channel. */
void or_pot_eval(const double p[7], double x, double y, double val[5],
                 double mag[5])
{
    double x0 = p[0], y0 = p[1], b0 = p[2], eps = p[3], phi = p[4];
    double a = p[5], s = p[6];
    double dx = x - x0, dy = y - y0;
    int k;
    if (a == 0.0 && dx == 0.0 && dy == 0.0) {
        for (k = 0; k < 5; k++) {
            val[k] = 0.0;
            if (mag) mag[k] = 0.0;
        }
        return;
    }
    double c = cos(phi), sn = sin(phi);
    double xp = dx * c + dy * sn;
    double yp = -dx * sn + dy * c;
    double Pa[5], Ps[5] = {0, 0, 0, 0, 0}, F = 1.0;
    cie_core(b0, eps, a, xp, yp, Pa);
    if (isfinite(s)) {
        cie_core(b0, eps, s, xp, yp, Ps);
        F = s / (s - a);
    }
    double d[5], ra[5], rs[5];
    for (k = 0; k < 5; k++) d[k] = F * (Pa[k] - Ps[k]);
    rotate_back(c, sn, d, val);
    if (mag) {
        rotate_back_abs(c, sn, Pa, ra);
        rotate_back_abs(c, sn, Ps, rs);
        for (k = 0; k < 5; k++) mag[k] = F * (ra[k] + rs[k]);
    }
}

/* Sum over n potentials (SoA arrays), in index order, at one point. */
typedef struct {
    int n;
    const double *x0, *y0, *b0, *eps, *phi, *rcore, *rcut;
} or_pots_t;

static void pots_sum(const or_pots_t *P, int lo, int hi, double x, double y,
                     double acc[5], double macc[5])
{
    int k, c;
    for (k = lo; k < hi; k++) {
        double p[7] = {P->x0[k], P->y0[k], P->b0[k], P->eps[k], P->phi[k],
                       P->rcore[k], P->rcut[k]};
        double v[5], m[5];
        or_pot_eval(p, x, y, v, macc ? m : NULL);
        for (c = 0; c < 5; c++) {
            acc[c] += v[c];
            if (macc) macc[c] += m[c];
        }
    }
}

/* Values at arbitrary points: out[c*npts + t] = sum_k (channel c of potential
 * k at point t), Dls/Ds = 1.  mag likewise (may be NULL). */
void or_eval_points(const or_pots_t *P, int npts, const double *x,
                    const double *y, double *out, double *mag)
{
    int t;
#pragma omp parallel for schedule(static)
    for (t = 0; t < npts; t++) {
        double acc[5] = {0, 0, 0, 0, 0}, macc[5] = {0, 0, 0, 0, 0};
        int c;
        pots_sum(P, 0, P->n, x[t], y[t], acc, mag ? macc : NULL);
        for (c = 0; c < 5; c++) {
            out[(size_t)c * npts + t] = acc[c];
            if (mag) mag[(size_t)c * npts + t] = macc[c];
        }
    }
}

/* Grid point (i, j) = (gx0 + i*dx, gy0 + j*dy): one product, one sum. */
static double grid_coord(double o, int i, double d) { return o + (double)i * d; }

/* Lensing map (Sec. 4.1, Eq. (10); Sec. 2.4): five planes, row-major
 * [ny][nx], out[c*nx*ny + j*nx + i] = dlsds * sum_k channel c.  mag gets the
 * matching condition scale (may be NULL).  OpenMP splits rows only; each
 * pixel's sum runs over k in index order. */
void or_map(const or_pots_t *P, int nx, int ny, double gx0, double gy0,
            double dx, double dy, double dlsds, double *out, double *mag)
{
    size_t np = (size_t)nx * ny;
    int j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < ny; j++) {
        int i, c;
        for (i = 0; i < nx; i++) {
            double acc[5] = {0, 0, 0, 0, 0}, macc[5] = {0, 0, 0, 0, 0};
            double x = grid_coord(gx0, i, dx), y = grid_coord(gy0, j, dy);
            pots_sum(P, 0, P->n, x, y, acc, mag ? macc : NULL);
            for (c = 0; c < 5; c++) {
                out[c * np + (size_t)j * nx + i] = dlsds * acc[c];
                if (mag) mag[c * np + (size_t)j * nx + i] = dlsds * macc[c];
            }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Lensing potential (Sec. 2.1: alpha = grad psi; one of the lensing maps of  */
/* Sec. 2.4) of one cored isothermal ellipsoid, in its own frame: the Keeton  */
/* (2001) softened-isothermal-ellipsoid form under the same mapping as the    */
/* deflection,                                                                */
/*   P_w = x' a'x + y' a'y - b0 (1 - eps^2) w ln sqrt((psi_w + S_w)^2 + k^2 x'^2) */
/* (circular: P_w = b0 [psi_w - w - w ln(psi_w + w)]), defined up to an       */
/* additive constant, which is fixed by this form.  mag receives the sum of   */
/* the magnitudes of its three terms.                                         */
/* ------------------------------------------------------------------------- */
static double cie_potential(double b0, double eps, double w, double xp, double yp,
                            double *mag)
{
    double q = (1.0 - eps) / (1.0 + eps);
    double q2 = q * q;
    double S = (1.0 + eps) * w;
    double pw = sqrt(q2 * (S * S + xp * xp) + yp * yp);  /* psi_w */
    double tx, ty, tl;
    if (eps > 0.0) {
        double k = 2.0 * sqrt(eps) / (1.0 + eps);
        double pref = b0 * (1.0 - eps * eps) / (2.0 * sqrt(eps));
        tx = xp * (pref * atan(k * xp / (pw + S)));
        ty = yp * (pref * atanh(k * yp / (pw + q2 * S)));
        tl = w > 0.0 ? b0 * (1.0 - eps * eps) * w * 0.5 *
                           log((pw + S) * (pw + S) + k * k * xp * xp)
                     : 0.0;
    } else {
        tx = xp * (b0 * xp / (pw + w));
        ty = yp * (b0 * yp / (pw + w));
        tl = w > 0.0 ? b0 * w * log(pw + w) : 0.0;
    }
    if (mag) *mag = fabs(tx) + fabs(ty) + fabs(tl);
    return tx + ty - tl;
}

/* dPIE potential p at (x, y), Dls/Ds = 1: F (P_a - P_s) (rcut = inf: F = 1,
 * no P_s); zero at the centre of a potential with rcore = 0 (its limit).
 * mag (may be NULL) receives F (mag_a + mag_s). */
double or_potential(const double p[7], double x, double y, double *mag)
{
    double x0 = p[0], y0 = p[1], b0 = p[2], eps = p[3], phi = p[4];
    double a = p[5], s = p[6];
    double dx = x - x0, dy = y - y0;
    if (a == 0.0 && dx == 0.0 && dy == 0.0) {
        if (mag) *mag = 0.0;
        return 0.0;
    }
    double c = cos(phi), sn = sin(phi);
    double xp = dx * c + dy * sn;
    double yp = -dx * sn + dy * c;
    double ma = 0.0, ms = 0.0, Ps = 0.0, F = 1.0;
    double Pa = cie_potential(b0, eps, a, xp, yp, &ma);
    if (isfinite(s)) {
        Ps = cie_potential(b0, eps, s, xp, yp, &ms);
        F = s / (s - a);
    }
    if (mag) *mag = F * (ma + ms);
    return F * (Pa - Ps);
}

/* Potential map (Dls/Ds scaling as for the deflection) and, with scale != 0,
 * the time-delay surface t = scale (|theta - beta|^2 / 2 - psi) of a source
 * at beta (Fermat potential; its stationary points are the images).
 * out, mag: ny*nx row-major (mag may be NULL; for t it bounds scale*psi). */
void or_potential_map(const or_pots_t *P, int nx, int ny, double gx0, double gy0,
                      double dx, double dy, double dlsds, double bx, double by,
                      double scale, double *out, double *mag)
{
    int j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < ny; j++) {
        int i, k;
        for (i = 0; i < nx; i++) {
            double x = grid_coord(gx0, i, dx), y = grid_coord(gy0, j, dy);
            double acc = 0.0, macc = 0.0, m;
            for (k = 0; k < P->n; k++) {
                double p[7] = {P->x0[k], P->y0[k], P->b0[k], P->eps[k], P->phi[k],
                               P->rcore[k], P->rcut[k]};
                acc += or_potential(p, x, y, &m);
                macc += m;
            }
            size_t at = (size_t)j * nx + i;
            if (scale != 0.0) {
                double ex = x - bx, ey = y - by;
                out[at] = scale * (0.5 * (ex * ex + ey * ey) - dlsds * acc);
                if (mag) mag[at] = fabs(scale) * (0.5 * (ex * ex + ey * ey) + dlsds * macc);
            } else {
                out[at] = dlsds * acc;
                if (mag) mag[at] = dlsds * macc;
            }
        }
    }
}

/* Time-delay scale (1 + zl) Dl Ds / (c Dls) in days per arcsec^2 for a flat
 * cosmology with H0 [km/s/Mpc]: the angular-diameter distances are
 * (c/H0) chi/(1+z) (Dls = (c/H0)(chi_s - chi_l)/(1+zs)), so the scale is
 * chi_l chi_s / ((chi_s - chi_l) H0) seconds per rad^2. */
static double comoving(double z, double om, double ol);
double or_time_delay_scale(double zl, double zs, double h0, double om, double ol)
{
    double cl = comoving(zl, om, ol), cs = comoving(zs, om, ol);
    double h0_si = h0 * 1000.0 / 3.0856775814913673e22;
    double rad = M_PI / 648000.0;
    return cl * cs / ((cs - cl) * h0_si) * rad * rad / 86400.0;
}

/* ------------------------------------------------------------------------- */
/* Derived maps from the summed second derivatives H (already scaled by      */
/* Dls/Ds).  Sec. 2.4, Eqs. (7)-(9) with Sec. 2.1's magnification matrix     */
/* A^-1 = [[1 - kappa - gamma1, -gamma2], [-gamma2, 1 - kappa + gamma1]]:    */
/*   kappa  = (Hxx + Hyy) / 2        (half the Laplacian, Eq. (7))           */
/*   gamma1 = (Hxx - Hyy) / 2, gamma2 = Hxy, gamma = sqrt(gamma1^2+gamma2^2) */
/*            (the shear of the summed Hessian; Eq. (8) read this way)        */
/*   det    = (1 - kappa)^2 - gamma^2  (the determinant of A^-1)              */
/*   mu     = 1 / det                  (Sec. 2.1; Eq. (9)'s "+" read as "-")  */
/* ------------------------------------------------------------------------- */
void or_derived(long n, const double *hxx, const double *hxy, const double *hyy,
                double *kappa, double *gamma1, double *gamma2, double *gamma,
                double *det, double *mu)
{
    long i;
    for (i = 0; i < n; i++) {
        double k = 0.5 * (hxx[i] + hyy[i]);
        double g1 = 0.5 * (hxx[i] - hyy[i]);
        double g2 = hxy[i];
        double gg = g1 * g1 + g2 * g2;
        double d = (1.0 - k) * (1.0 - k) - gg;
        kappa[i] = k;
        gamma1[i] = g1;
        gamma2[i] = g2;
        gamma[i] = sqrt(gg);
        det[i] = d;
        mu[i] = 1.0 / d;
    }
}

/* ------------------------------------------------------------------------- */
/* Distance ratio Dls/Ds (Sec. 2.1, Eq. (3)).  Flat LCDM: comoving distance   */
/* chi(z) = int_0^z dz'/E(z'), E = sqrt(om (1+z)^3 + ol); Dls/Ds =             */
/* 1 - chi(zl)/chi(zs).  Composite Simpson rule, 20000 panels.                */
/* ------------------------------------------------------------------------- */
static double inv_E(double z, double om, double ol)
{
    double a = 1.0 + z;
    return 1.0 / sqrt(om * a * a * a + ol);
}

static double comoving(double z, double om, double ol)
{
    const int n = 20000; /* even */
    double h = z / n, s = inv_E(0.0, om, ol) + inv_E(z, om, ol);
    int i;
    for (i = 1; i < n; i++) s += (i % 2 ? 4.0 : 2.0) * inv_E(i * h, om, ol);
    return s * h / 3.0;
}

/* Returns 0 and *out, or -1 when zs <= zl, zl < 0 or the model is not flat. */
int or_dlsds(double zl, double zs, double om, double ol, double *out)
{
    if (!(zl >= 0.0) || !(zs > zl) || !(om >= 0.0) || !(ol >= 0.0) ||
        fabs(om + ol - 1.0) > 1e-9)
        return -1;
    *out = 1.0 - comoving(zl, om, ol) / comoving(zs, om, ol);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Source-plane chi^2 (Sec. 2.2, Eq. (6) and Fig. 3).                         */
/* ------------------------------------------------------------------------- */
typedef struct {
    int nsys;
    const int *off;        /* [nsys+1] image offsets */
    const double *x, *y;   /* observed image positions c_ij */
    const double *sig;     /* sigma_ij */
    const double *f;       /* Dls/Ds of each system */
} or_cat_t;

/* Deflection at one point for model m: fixed potentials then the free
 * potentials of sample m, all in index order (Dls/Ds = 1).  mag: |.| sum. */
static void model_alpha(const or_pots_t *fixed, const or_pots_t *freep,
                        const int *free_off, int m, double x, double y,
                        double a[2], double am[2])
{
    double acc[5] = {0, 0, 0, 0, 0}, macc[5] = {0, 0, 0, 0, 0};
    pots_sum(fixed, 0, fixed->n, x, y, acc, am ? macc : NULL);
    pots_sum(freep, free_off[m], free_off[m + 1], x, y, acc, am ? macc : NULL);
    a[0] = acc[0];
    a[1] = acc[1];
    if (am) {
        am[0] = macc[0];
        am[1] = macc[1];
    }
}

/* Unlensed positions beta_ij = theta_ij - f_i alpha(theta_ij) of every image
 * for sample m.  sabs[t] (may be NULL) = |alpha_x| + |alpha_y| terms bound. */
void or_unlens(const or_pots_t *fixed, const or_pots_t *freep,
               const int *free_off, int m, const or_cat_t *C, double *bx,
               double *by, double *sabs)
{
    int i, t;
    for (i = 0; i < C->nsys; i++) {
        for (t = C->off[i]; t < C->off[i + 1]; t++) {
            double a[2], am[2];
            model_alpha(fixed, freep, free_off, m, C->x[t], C->y[t], a,
                        sabs ? am : NULL);
            bx[t] = C->x[t] - C->f[i] * a[0];
            by[t] = C->y[t] - C->f[i] * a[1];
            if (sabs) sabs[t] = am[0] + am[1];
        }
    }
}

/* Barycentre of the unlensed images of each system (Sec. 2.2): mean of
 * beta_ij over j.  Systems without images get (0, 0). */
static void barycentres(const or_cat_t *C, const double *bx, const double *by,
                        double *sx, double *sy)
{
    int i, t;
    for (i = 0; i < C->nsys; i++) {
        int M = C->off[i + 1] - C->off[i];
        double mx = 0.0, my = 0.0;
        for (t = C->off[i]; t < C->off[i + 1]; t++) {
            mx += bx[t];
            my += by[t];
        }
        sx[i] = M > 0 ? mx / M : 0.0;
        sy[i] = M > 0 ? my / M : 0.0;
    }
}

/* chi2[m] = sum_i sum_j |beta_ij - bar beta_i|^2 / sigma_ij^2, one sample
 * after another; OpenMP over samples only. */
void or_chi2_source(const or_pots_t *fixed, const or_pots_t *freep,
                    const int *free_off, int nsamp, const or_cat_t *C,
                    double *chi2)
{
    int nimg = C->off[C->nsys];
    int m;
#pragma omp parallel for schedule(dynamic)
    for (m = 0; m < nsamp; m++) {
        double *bx = malloc(sizeof(double) * (nimg + 1));
        double *by = malloc(sizeof(double) * (nimg + 1));
        double *sx = malloc(sizeof(double) * (C->nsys + 1));
        double *sy = malloc(sizeof(double) * (C->nsys + 1));
        double total = 0.0;
        int i, t;
        or_unlens(fixed, freep, free_off, m, C, bx, by, NULL);
        barycentres(C, bx, by, sx, sy);
        for (i = 0; i < C->nsys; i++) {
            double part = 0.0;
            for (t = C->off[i]; t < C->off[i + 1]; t++) {
                double ex = bx[t] - sx[i], ey = by[t] - sy[i];
                part += (ex * ex + ey * ey) / (C->sig[t] * C->sig[t]);
            }
            total += part;
        }
        chi2[m] = total;
        free(bx);
        free(by);
        free(sx);
        free(sy);
    }
}

/* Barycentric sources of sample m (the source step of Sec. 4.2). */
void or_sources(const or_pots_t *fixed, const or_pots_t *freep,
                const int *free_off, int m, const or_cat_t *C, double *sx,
                double *sy)
{
    int nimg = C->off[C->nsys];
    double *bx = malloc(sizeof(double) * (nimg + 1));
    double *by = malloc(sizeof(double) * (nimg + 1));
    or_unlens(fixed, freep, free_off, m, C, bx, by, NULL);
    barycentres(C, bx, by, sx, sy);
    free(bx);
    free(by);
}

/* ------------------------------------------------------------------------- */
/* Exact orientation sign.                                                    */
/* orient(a, b, p) = (bx-ax)(py-ay) - (by-ay)(px-ax) expands to the six exact */
/* products +bx*py -bx*ay -ax*py -by*px +by*ax +ay*px (the ax*ay terms        */
/* cancel).  Each double is an integer times a power of two, so the sum is an */
/* exact integer in a wide fixed-point accumulator; its sign is exact.        */
/* ------------------------------------------------------------------------- */
#define OR_NL 142           /* 32-bit limbs (4544 bits) */
#define OR_BIAS 2260        /* bit index of the accumulator's 2^0 */

static void split_double(double d, uint64_t *m, int *e, int *neg)
{
    int E;
    double f;
    if (d == 0.0) {
        *m = 0;
        *e = 0;
        *neg = 0;
        return;
    }
    f = frexp(fabs(d), &E);            /* |d| = f 2^E, 1/2 <= f < 1 */
    *m = (uint64_t)ldexp(f, 53);       /* integer: d has <= 53 significant bits */
    *e = E - 53;
    *neg = d < 0.0;
}

static void acc_product(int64_t *L, double u, double v, int sign)
{
    uint64_t mu, mv;
    int eu, ev, nu, nv, t;
    split_double(u, &mu, &eu, &nu);
    split_double(v, &mv, &ev, &nv);
    if (mu == 0 || mv == 0) return;
    unsigned __int128 M = (unsigned __int128)mu * mv; /* < 2^106 */
    int pos = eu + ev + OR_BIAS;                       /* >= 0 */
    int limb = pos >> 5, sh = pos & 31;
    int neg = (nu ^ nv) ^ (sign < 0);
    for (t = 0; t < 4; t++) {
        uint64_t chunk = (uint64_t)(M >> (32 * t)) & 0xffffffffull;
        uint64_t w = chunk << sh;                          /* < 2^63 */
        int64_t lo = (int64_t)(w & 0xffffffffull), hi = (int64_t)(w >> 32);
        if (neg) {
            lo = -lo;
            hi = -hi;
        }
        L[limb + t] += lo;
        L[limb + t + 1] += hi;
    }
}

static int acc_sign(int64_t *L)
{
    const int64_t B = 4294967296LL;
    int64_t carry = 0;
    int i, nz = 0;
    for (i = 0; i < OR_NL; i++) {
        int64_t v = L[i] + carry;
        int64_t q = v >= 0 ? v / B : -((-v + B - 1) / B); /* floor(v / B) */
        L[i] = v - q * B;                                 /* in [0, B) */
        carry = q;
        if (L[i]) nz = 1;
    }
    if (carry < 0) return -1;
    if (carry > 0) return 1;
    return nz;
}

int or_orient_exact(double ax, double ay, double bx, double by, double px,
                    double py)
{
    /* Fast answer when the rounded value is far from zero.  The rounding error
     * of this expression is below 4e-16 (|l| + |r|) (Shewchuk 1997), so a
     * margin of 1e-12 (|l| + |r|) leaves the sign certain. */
    double l = (bx - ax) * (py - ay), r = (by - ay) * (px - ax);
    double det = l - r, sum = fabs(l) + fabs(r);
    if (sum > 1e-250 && sum < 1e250 && fabs(det) > 1e-12 * sum)
        return det > 0.0 ? 1 : -1;
    int64_t L[OR_NL];
    memset(L, 0, sizeof L);
    acc_product(L, bx, py, +1);
    acc_product(L, bx, ay, -1);
    acc_product(L, ax, py, -1);
    acc_product(L, by, px, -1);
    acc_product(L, by, ax, +1);
    acc_product(L, ay, px, +1);
    return acc_sign(L);
}

/* Sign of orient(a, b, p + (d, d^2)) for an infinitesimal d > 0: the exact
 * sign if nonzero, else the sign of -(by-ay), else the sign of (bx-ax). */
int or_orient_perturbed(double ax, double ay, double bx, double by, double px,
                        double py)
{
    int s = or_orient_exact(ax, ay, bx, by, px, py);
    if (s) return s;
    if (by != ay) return by < ay ? 1 : -1;
    if (bx != ax) return bx > ax ? 1 : -1;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Brute-force image search on the triangulated grid (Sec. 2.3, Fig. 4).      */
/* ------------------------------------------------------------------------- */
/* Refinement of one found image (Sec. 2.3: a found image is refined until a  */
/* set precision is reached; the paper subdivides the containing triangle     */
/* recursively).  This oracle solves the lens equation beta = theta - f alpha */
/* (Sec. 2.1, Eq. (1)) for theta near the grid estimate by Newton's method    */
/* with the analytic second derivatives (Sec. 2.4):                           */
/*   r = beta - (theta - f alpha(theta)),  A = I - f H(theta),               */
/*   theta <- theta + A^-1 r,                                                 */
/* stopping when the step is shorter than tol.  alpha and H sum the fixed     */
/* potentials then the sample's free ones (index order).  Returns the number  */
/* of iterations, or -1 when the iteration does not converge within max_iter  */
/* or leaves the box |theta - theta0| <= max_shift (each coordinate); the     */
/* input position is then kept.                                               */
/* ------------------------------------------------------------------------- */
int or_refine_image(const or_pots_t *fixed, const or_pots_t *freep, int k0, int k1,
                    double f, double bx, double by, double *x, double *y,
                    int max_iter, double tol, double max_shift)
{
    double x0 = *x, y0 = *y, cx = *x, cy = *y;
    int it;
    for (it = 0; it < max_iter; it++) {
        double acc[5] = {0, 0, 0, 0, 0};
        double rx, ry, a11, a12, a22, det, sx, sy;
        pots_sum(fixed, 0, fixed->n, cx, cy, acc, NULL);
        pots_sum(freep, k0, k1, cx, cy, acc, NULL);
        rx = bx - (cx - f * acc[0]);
        ry = by - (cy - f * acc[1]);
        a11 = 1.0 - f * acc[2];
        a12 = -(f * acc[3]);
        a22 = 1.0 - f * acc[4];
        det = a11 * a22 - a12 * a12;
        sx = (a22 * rx - a12 * ry) / det;
        sy = (a11 * ry - a12 * rx) / det;
        cx = cx + sx;
        cy = cy + sy;
        if (!(fabs(cx - x0) <= max_shift && fabs(cy - y0) <= max_shift)) return -1;
        if (sx * sx + sy * sy < tol * tol) {
            *x = cx;
            *y = cy;
            return it + 1;
        }
    }
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Cell (i, j), 0 <= i < nx-1, 0 <= j < ny-1, is split into
 *   T0 = (v[i,j], v[i+1,j], v[i,j+1])  and  T1 = (v[i+1,j+1], v[i,j+1], v[i+1,j]),
 * with triangle ids 2 (j (nx-1) + i) and that + 1.  Each vertex maps to the
 * source plane as u = v - f alpha(v) (one product, one difference).  The source
 * p lies in a triangle when the three perturbed edge orientations agree;
 * triangles of exactly zero source-plane area are skipped.  The image is the
 * barycentric interpolation of the image-plane vertices with weights
 * o_a = orient(u_b, u_c, p), o_b = orient(u_c, u_a, p), o_c = orient(u_a, u_b, p).
 * Images come out in increasing triangle id.  Returns the exact number of
 * containing triangles; only the first kmax are stored. */
int or_find_images(const double *ax, const double *ay, int nx, int ny,
                   double gx0, double gy0, double dx, double dy, double f,
                   double px, double py, int kmax, long long *tri,
                   double *ix, double *iy)
{
    int n = 0, i, j, t;
    for (j = 0; j + 1 < ny; j++) {
        for (i = 0; i + 1 < nx; i++) {
            for (t = 0; t < 2; t++) {
                int vi[3], vj[3], k;
                double vx[3], vy[3], ux[3], uy[3];
                if (t == 0) {
                    vi[0] = i;     vj[0] = j;
                    vi[1] = i + 1; vj[1] = j;
                    vi[2] = i;     vj[2] = j + 1;
                } else {
                    vi[0] = i + 1; vj[0] = j + 1;
                    vi[1] = i;     vj[1] = j + 1;
                    vi[2] = i + 1; vj[2] = j;
                }
                for (k = 0; k < 3; k++) {
                    size_t id = (size_t)vj[k] * nx + vi[k];
                    vx[k] = grid_coord(gx0, vi[k], dx);
                    vy[k] = grid_coord(gy0, vj[k], dy);
                    ux[k] = vx[k] - f * ax[id];
                    uy[k] = vy[k] - f * ay[id];
                }
                if (or_orient_exact(ux[0], uy[0], ux[1], uy[1], ux[2], uy[2]) == 0)
                    continue;
                int s0 = or_orient_perturbed(ux[0], uy[0], ux[1], uy[1], px, py);
                int s1 = or_orient_perturbed(ux[1], uy[1], ux[2], uy[2], px, py);
                int s2 = or_orient_perturbed(ux[2], uy[2], ux[0], uy[0], px, py);
                if (!(s0 == s1 && s1 == s2 && s0 != 0)) continue;
                if (n < kmax) {
                    double oa = (ux[2] - ux[1]) * (py - uy[1]) - (uy[2] - uy[1]) * (px - ux[1]);
                    double ob = (ux[0] - ux[2]) * (py - uy[2]) - (uy[0] - uy[2]) * (px - ux[2]);
                    double oc = (ux[1] - ux[0]) * (py - uy[0]) - (uy[1] - uy[0]) * (px - ux[0]);
                    double den = (oa + ob) + oc;
                    if (den != 0.0) {
                        ix[n] = ((oa * vx[0] + ob * vx[1]) + oc * vx[2]) / den;
                        iy[n] = ((oa * vy[0] + ob * vy[1]) + oc * vy[2]) / den;
                    } else {
                        ix[n] = ((vx[0] + vx[1]) + vx[2]) / 3.0;
                        iy[n] = ((vy[0] + vy[1]) + vy[2]) / 3.0;
                    }
                    tri[n] = 2LL * ((long long)j * (nx - 1) + i) + t;
                }
                n++;
            }
        }
    }
    return n;
}

/* Assignment and chi^2 of one system (Sec. 4.2: found images go to their
 * closest constraint, then Eq. (6)).  Each stored image picks its nearest
 * constraint (ties: lower constraint index); each constraint keeps the nearest
 * image it was picked by (ties: lower triangle id, i.e. earlier in the list).
 * Constraints left without an image add `penalty` and count as missing.
 * Distances are ((x-cx)^2 + (y-cy)^2) in plain FP64. */
double or_assign_system(int nimg, const double *ix, const double *iy, int M,
                        const double *cx, const double *cy, const double *sig,
                        double penalty, int *nmissing)
{
    double part = 0.0;
    int j, k, miss = 0;
    int *pick = malloc(sizeof(int) * (nimg + 1));
    for (k = 0; k < nimg; k++) {
        double best = 0.0;
        int bj = -1;
        for (j = 0; j < M; j++) {
            double ex = ix[k] - cx[j], ey = iy[k] - cy[j];
            double d2 = ex * ex + ey * ey;
            if (bj < 0 || d2 < best) {
                best = d2;
                bj = j;
            }
        }
        pick[k] = bj;
    }
    for (j = 0; j < M; j++) {
        double best = 0.0;
        int found = 0;
        for (k = 0; k < nimg; k++) {
            if (pick[k] != j) continue;
            double ex = ix[k] - cx[j], ey = iy[k] - cy[j];
            double d2 = ex * ex + ey * ey;
            if (!found || d2 < best) {
                best = d2;
                found = 1;
            }
        }
        if (found)
            part += best / (sig[j] * sig[j]);
        else {
            part += penalty;
            miss++;
        }
    }
    free(pick);
    *nmissing = miss;
    return part;
}

/* Image-plane chi^2 of samples [m0, m1) (Sec. 4.2, the four stages):
 *   (1) deflection at every grid vertex: alpha_fix (the fixed potentials,
 *       summed in index order, Dls/Ds = 1, given) plus the free potentials of
 *       the sample, added in index order;
 *   (2) barycentric sources from the constraints;
 *   (3) brute-force image search per system;
 *   (4) assignment and chi^2.
 * Outputs, per sample s = m - m0: chi2[s]; nimg[s*nsys + i]; nmiss[s];
 * img_x/img_y/img_tri[(s*nsys + i)*kmax + k] for the stored images (may be
 * NULL).  Returns the number of (sample, system) pairs whose image count
 * exceeded kmax.  OpenMP over vertices and systems; every per-item result is
 * computed independently of the split. */
int or_chi2_image(const or_pots_t *fixed, const or_pots_t *freep,
                  const int *free_off, int m0, int m1, const or_cat_t *C,
                  const double *alpha_fix_x, const double *alpha_fix_y, int nx,
                  int ny, double gx0, double gy0, double dx, double dy,
                  int kmax, double penalty, double *chi2, int *nimg,
                  int *nmiss, double *img_x, double *img_y,
                  long long *img_tri, int refine_max_iter, double refine_tol,
                  double refine_max_shift, int *nfail)
{
    size_t nv = (size_t)nx * ny;
    double *gax = malloc(sizeof(double) * nv), *gay = malloc(sizeof(double) * nv);
    double *sx = malloc(sizeof(double) * (C->nsys + 1));
    double *sy = malloc(sizeof(double) * (C->nsys + 1));
    double *part = malloc(sizeof(double) * (C->nsys + 1));
    int *miss = malloc(sizeof(int) * (C->nsys + 1));
    int over = 0, m;
    for (m = m0; m < m1; m++) {
        int s = m - m0, i;
        long v;
#pragma omp parallel for schedule(static)
        for (v = 0; v < (long)nv; v++) {
            double acc[5] = {alpha_fix_x[v], alpha_fix_y[v], 0, 0, 0};
            int ii = (int)(v % nx), jj = (int)(v / nx);
            pots_sum(freep, free_off[m], free_off[m + 1], grid_coord(gx0, ii, dx),
                     grid_coord(gy0, jj, dy), acc, NULL);
            gax[v] = acc[0];
            gay[v] = acc[1];
        }
        or_sources(fixed, freep, free_off, m, C, sx, sy);
        int fails = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : over, fails)
        for (i = 0; i < C->nsys; i++) {
            int cap = kmax > 0 ? kmax : 0;
            long long *tri = malloc(sizeof(long long) * (cap + 1));
            double *ix = malloc(sizeof(double) * (cap + 1));
            double *iy = malloc(sizeof(double) * (cap + 1));
            int n = or_find_images(gax, gay, nx, ny, gx0, gy0, dx, dy, C->f[i],
                                   sx[i], sy[i], cap, tri, ix, iy);
            int stored = n < cap ? n : cap, k;
            if (n > cap) over++;
            if (refine_max_iter > 0)
                for (k = 0; k < stored; k++)
                    if (or_refine_image(fixed, freep, free_off[m], free_off[m + 1], C->f[i],
                                        sx[i], sy[i], &ix[k], &iy[k], refine_max_iter,
                                        refine_tol, refine_max_shift) < 0)
                        fails++;
            int o = C->off[i], M = C->off[i + 1] - C->off[i];
            part[i] = or_assign_system(stored, ix, iy, M, C->x + o, C->y + o,
                                       C->sig + o, penalty, &miss[i]);
            if (nimg) nimg[(size_t)s * C->nsys + i] = n;
            for (k = 0; k < stored; k++) {
                size_t at = ((size_t)s * C->nsys + i) * cap + k;
                if (img_x) img_x[at] = ix[k];
                if (img_y) img_y[at] = iy[k];
                if (img_tri) img_tri[at] = tri[k];
            }
            free(tri);
            free(ix);
            free(iy);
        }
        double total = 0.0;
        int nm = 0;
        for (i = 0; i < C->nsys; i++) {
            total += part[i];
            nm += miss[i];
        }
        chi2[s] = total;
        if (nmiss) nmiss[s] = nm;
        if (nfail) nfail[s] = fails;
    }
    free(gax);
    free(gay);
    free(sx);
    free(sy);
    free(part);
    free(miss);
    return over;
}

/* ------------------------------------------------------------------------- */
/* One step of a Metropolis sampler over the free potentials' physical        */
/* parameters (Sec. 2.2: the parameter space is explored by a Bayesian MCMC;  */
/* Sec. 4 names the sampler the third bottleneck).  Walker w holds nfree      */
/* potentials of 7 parameters (x0, y0, sigma, e, phi, rcore, rcut) in         */
/* params[w][k][j]; u[w][0 .. 7 nfree] are uniforms in (0, 1] supplied by the */
/* caller.  Proposal: theta'_i = theta_i + step_i (2 u_i - 1) (symmetric);    */
/* a proposal outside the prior box [lo, hi] is rejected.  Otherwise it is    */
/* accepted when chi2' <= chi2 or -2 ln u_last > chi2' - chi2, i.e. with      */
/* probability min(1, exp(-(chi2' - chi2)/2)) for the likelihood exp(-chi2/2) */
/* and uniform priors.  chi2' is the source-plane chi^2 (fixed potentials     */
/* then the walker's, in index order; sigma -> b0 and e -> eps as the         */
/* parameter conversions below).  Returns the number of accepted moves.       */
/* ------------------------------------------------------------------------- */
double or_b0_from_sigma(double sigma_kms, int convention);
double or_eps_from_e(double e);

int or_mcmc_step(const or_pots_t *fixed, const or_cat_t *C, int W, int nfree,
                 double *params, double *chi2, int *accepted, const double *lo,
                 const double *hi, const double *step, const double *u, int convention)
{
    int P = 7 * nfree, w, i, k, acc = 0;
    double *prop = malloc(sizeof(double) * ((size_t)W * P + 1));
    double *amp = malloc(sizeof(double) * ((size_t)7 * W * nfree + 1));
    double *chi2p = malloc(sizeof(double) * (W + 1));
    int *inside = malloc(sizeof(int) * (W + 1));
    int *off = malloc(sizeof(int) * (W + 1));
    size_t n = (size_t)W * nfree;
    for (w = 0; w < W; w++) {
        const double *th = params + (size_t)w * P;
        const double *uw = u + (size_t)w * (P + 1);
        double *pr = prop + (size_t)w * P;
        int in = 1;
        for (i = 0; i < P; i++) {
            pr[i] = th[i] + step[i] * (2.0 * uw[i] - 1.0);
            if (!(pr[i] >= lo[i] && pr[i] <= hi[i])) in = 0;
        }
        inside[w] = in;
        off[w] = w * nfree;
        /* an out-of-prior proposal is never evaluated: its slot holds the
           current (valid) parameters */
        const double *src = in ? pr : th;
        for (k = 0; k < nfree; k++) {
            size_t at = (size_t)w * nfree + k;
            const double *q = src + 7 * k;
            amp[0 * n + at] = q[0];
            amp[1 * n + at] = q[1];
            amp[2 * n + at] = or_b0_from_sigma(q[2], convention);
            amp[3 * n + at] = or_eps_from_e(q[3]);
            amp[4 * n + at] = q[4];
            amp[5 * n + at] = q[5];
            amp[6 * n + at] = q[6];
        }
    }
    off[W] = W * nfree;
    or_pots_t freep = {(int)n, amp, amp + n, amp + 2 * n, amp + 3 * n, amp + 4 * n,
                       amp + 5 * n, amp + 6 * n};
    or_chi2_source(fixed, &freep, off, W, C, chi2p);
    for (w = 0; w < W; w++) {
        double d = chi2p[w] - chi2[w];
        double ul = u[(size_t)w * (P + 1) + P];
        if (inside[w] && (d <= 0.0 || -2.0 * log(ul) > d)) {
            memcpy(params + (size_t)w * P, prop + (size_t)w * P, sizeof(double) * P);
            chi2[w] = chi2p[w];
            accepted[w] += 1;
            acc++;
        }
    }
    free(prop);
    free(amp);
    free(chi2p);
    free(inside);
    free(off);
    return acc;
}

/* Smallest distance from p to any triangle edge (segment) of the unlensed grid
 * for one system.  A containment decision can only differ between two
 * evaluations whose vertex and source positions differ by less than this. */
double or_edge_margin(const double *ax, const double *ay, int nx, int ny,
                      double gx0, double gy0, double dx, double dy, double f,
                      double px, double py)
{
    double best = INFINITY;
    int i, j, e;
    for (j = 0; j < ny; j++) {
        for (i = 0; i < nx; i++) {
            /* edges from v[i,j] to its right, upper and upper-left neighbours
             * cover every triangle edge of the T0/T1 split exactly once */
            int ni[3] = {i + 1, i, i + 1}, nj[3] = {j, j + 1, j + 1};
            size_t id = (size_t)j * nx + i;
            double x1 = grid_coord(gx0, i, dx) - f * ax[id];
            double y1 = grid_coord(gy0, j, dy) - f * ay[id];
            for (e = 0; e < 3; e++) {
                int i2 = ni[e], j2 = nj[e];
                if (e == 2) { /* diagonal of cell (i, j): v[i+1,j] -- v[i,j+1] */
                    if (i + 1 >= nx || j + 1 >= ny) continue;
                    size_t ia = (size_t)j * nx + (i + 1), ib = (size_t)(j + 1) * nx + i;
                    double xa = grid_coord(gx0, i + 1, dx) - f * ax[ia];
                    double ya = grid_coord(gy0, j, dy) - f * ay[ia];
                    double xb = grid_coord(gx0, i, dx) - f * ax[ib];
                    double yb = grid_coord(gy0, j + 1, dy) - f * ay[ib];
                    double ex = xb - xa, ey = yb - ya, L2 = ex * ex + ey * ey;
                    double tt = L2 > 0 ? ((px - xa) * ex + (py - ya) * ey) / L2 : 0.0;
                    if (tt < 0) tt = 0;
                    if (tt > 1) tt = 1;
                    double qx = xa + tt * ex - px, qy = ya + tt * ey - py;
                    double dd = sqrt(qx * qx + qy * qy);
                    if (dd < best) best = dd;
                    continue;
                }
                if (i2 >= nx || j2 >= ny) continue;
                size_t id2 = (size_t)j2 * nx + i2;
                double x2 = grid_coord(gx0, i2, dx) - f * ax[id2];
                double y2 = grid_coord(gy0, j2, dy) - f * ay[id2];
                double ex = x2 - x1, ey = y2 - y1, L2 = ex * ex + ey * ey;
                double tt = L2 > 0 ? ((px - x1) * ex + (py - y1) * ey) / L2 : 0.0;
                if (tt < 0) tt = 0;
                if (tt > 1) tt = 1;
                double qx = x1 + tt * ex - px, qy = y1 + tt * ey - py;
                double dd = sqrt(qx * qx + qy * qy);
                if (dd < best) best = dd;
            }
        }
    }
    return best;
}

/* ------------------------------------------------------------------------- */
/* Physical parameters -> amplitude form.                                     */
/* ------------------------------------------------------------------------- */
/* Deflection amplitude at Dls/Ds = 1, in arcsec, from a velocity dispersion in
 * km/s: b0 = K pi (sigma/c)^2 rad, K = 6 for the Lenstool dPIE convention
 * (convention 0) and K = 4 for the singular isothermal sphere (convention 1). */
double or_b0_from_sigma(double sigma_kms, int convention)
{
    const double c_kms = 299792.458;
    const double rad_to_arcsec = 180.0 * 3600.0 / 3.14159265358979323846;
    double K = convention == 1 ? 4.0 : 6.0;
    double v = sigma_kms / c_kms;
    return K * 3.14159265358979323846 * v * v * rad_to_arcsec;
}

/* Kassiola-Kovner eps = (a-b)/(a+b) from the Lenstool e = (a^2-b^2)/(a^2+b^2):
 * eps = (1 - sqrt(1-e^2))/e, written as e/(1 + sqrt(1-e^2)) (no cancellation
 * at small e; eps = 0 at e = 0). */
double or_eps_from_e(double e) { return e / (1.0 + sqrt(1.0 - e * e)); }
