"""Shared helpers of the GPU parity tests: move seeded inputs to the device,
build the same model for the oracle, and compare under the stated tolerances.

Tolerances (per element, condition-scaled): |gpu - oracle| <= rtol * scale,
where scale is the oracle's sum over potentials of the magnitudes of the terms
each channel is built from (its `mag` output).  rtol = 1e-12 for FP64 and
1e-5 for the FP32 evaluation modes.
"""
import numpy as np

RTOL = {0: 1e-12, 1: 1e-5, 2: 1e-5}


def grid_points(grid, ii, jj):
    """Coordinates of grid points (one rounded product, one rounded sum)."""
    nx, ny, x0, y0, dx, dy = grid
    ii, jj = np.asarray(ii), np.asarray(jj)
    return x0 + ii.astype(np.float64) * dx, y0 + jj.astype(np.float64) * dy


def assert_within(got, ref, scale, rtol, what=""):
    got, ref, scale = (np.asarray(a, dtype=np.float64) for a in (got, ref, scale))
    err = np.abs(got - ref)
    bound = rtol * scale
    bad = ~(err <= bound)
    if bad.any():
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio = np.where(scale > 0, err / scale, np.inf)
        k = np.unravel_index(np.nanargmax(np.where(bad, ratio, -1)), err.shape)
        raise AssertionError(
            f"{what}: {int(bad.sum())} of {err.size} elements exceed rtol={rtol:g} * scale; "
            f"worst at {k}: got {got[k]!r} ref {ref[k]!r} scale {scale[k]!r} "
            f"(err/scale {ratio[k]:.3g})")
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(scale > 0, err / scale, 0.0)
    return float(np.max(r)) if r.size else 0.0


def chi2_source_bound(bx, by, sabs, cat, rtol):
    """Error bound of a source-plane chi^2 whose unlensed positions each carry
    an error up to e_ij = rtol (|theta_ij| + f_i sabs_ij): a residual
    d = beta_ij - mean_j beta then errs by at most 2 max_j e_ij =: D and the
    term |d|^2/sigma^2 by (2|d| D + D^2)/sigma^2."""
    off = np.asarray(cat["off"])
    total = 0.0
    for i in range(len(off) - 1):
        s = slice(off[i], off[i + 1])
        if off[i + 1] == off[i]:
            continue
        th = np.hypot(cat["x"][s], cat["y"][s])
        e = rtol * (th + cat["f"][i] * sabs[s])
        D = 2.0 * e.max() + 4e-16 * (th.max() + cat["f"][i] * sabs[s].max())
        mx, my = bx[s].mean(), by[s].mean()
        d = np.hypot(bx[s] - mx, by[s] - my)
        total += np.sum((2 * d * D + D * D) / cat["sig"][s] ** 2)
    return total


def derived_bounds(h, mag, rtol, stored_f32=False):
    """Per-element error bounds of the derived maps given second derivatives
    h = (hxx, hxy, hyy) that each err by at most rtol * mag (the map
    tolerance): first-order propagation through kappa, gamma1, gamma2,
    gamma, det = (1-kappa)^2 - gamma^2 plus the second-order terms, a few
    units of rounding of the formulas themselves, and one FP32 rounding of
    the stored value when the outputs are single precision.  mu is bounded
    only where |det| exceeds twice its bound (elsewhere it is NaN: not
    compared)."""
    e = 2.0 ** -52
    hxx, hxy, hyy = (np.asarray(v, dtype=np.float64) for v in h)
    dxx, dxy, dyy = (rtol * np.asarray(m, dtype=np.float64) for m in mag)
    k = 0.5 * (hxx + hyy)
    g1 = 0.5 * (hxx - hyy)
    g2 = hxy
    gg = g1 * g1 + g2 * g2
    om = 1.0 - k
    det = om * om - gg
    dk = 0.5 * (dxx + dyy) + 2 * e * np.abs(k)
    dg1 = 0.5 * (dxx + dyy) + 2 * e * np.abs(g1)
    dg2 = dxy
    dg = dg1 + dg2 + 4 * e * np.sqrt(gg)
    ddet = (2 * np.abs(om) * dk + dk * dk + 2 * np.abs(g1) * dg1 + dg1 * dg1
            + 2 * np.abs(g2) * dg2 + dg2 * dg2 + 8 * e * (om * om + gg))
    with np.errstate(divide="ignore", invalid="ignore"):
        ok = np.abs(det) > 2 * ddet
        mu = 1.0 / det
        dmu = np.where(ok, ddet / (np.abs(det) * (np.abs(det) - ddet)) + 4 * e * np.abs(mu), np.nan)
    out = dict(kappa=dk, gamma1=dg1, gamma2=dg2, gamma=dg, det=ddet, mu=dmu)
    if stored_f32:
        vals = dict(kappa=k, gamma1=g1, gamma2=g2, gamma=np.sqrt(gg), det=det, mu=mu)
        out = {n: b + np.abs(vals[n]) * 2.0 ** -24 for n, b in out.items()}
    return out
