"""Shared helpers of the GPU parity tests: move seeded inputs to the device,
build the same model for the oracle, and compare under the stated tolerances.

Tolerances (per element, condition-scaled): |gpu - oracle| <= rtol * scale,
where scale is the oracle's sum over potentials of the magnitudes of the terms
each channel is built from (its `mag` output).  rtol = 1e-12 for FP64 and
1e-5 for the FP32 evaluation modes.
"""
import math

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


# --------------------------------------------------------------------------
# Image-plane chi^2: error bounds derived from the deflection tolerance
# --------------------------------------------------------------------------
U = 2.0 ** -53  # unit roundoff of FP64


def tri_vertices(tri, grid):
    """Vertex indices (i, j) of triangle `tri` of the T0/T1 split: cell
    c = tri // 2 = j (nx - 1) + i; T0 = (v[i,j], v[i+1,j], v[i,j+1]),
    T1 = (v[i+1,j+1], v[i,j+1], v[i+1,j])."""
    c, t = divmod(int(tri), 2)
    j, i = divmod(c, grid[0] - 1)
    if t == 0:
        return [(i, j), (i + 1, j), (i, j + 1)]
    return [(i + 1, j + 1), (i, j + 1), (i + 1, j)]


def source_errors(bx, by, sabs, cat, rtol):
    """Bound on the error of each system's barycentric source when every
    deflection may err by rtol * scale: each unlensed position by at most
    rtol (|theta| + f sabs) per component (sabs = |.|x + |.|y scale of the
    image), so the mean by at most the largest of them (Euclidean: times
    sqrt 2), plus the rounding of the mean."""
    off = np.asarray(cat["off"])
    out = np.zeros(len(off) - 1)
    for i in range(len(off) - 1):
        s = slice(off[i], off[i + 1])
        if off[i + 1] == off[i]:
            continue
        th = np.hypot(cat["x"][s], cat["y"][s])
        e = math.sqrt(2.0) * rtol * (th + cat["f"][i] * sabs[s])
        out[i] = e.max() + 8 * U * np.hypot(bx[s], by[s]).max()
    return out


def _norm2(a, b, c, d):
    """Spectral norm of the 2x2 matrices [[a, b], [c, d]] (arrays)."""
    s = a * a + b * b + c * c + d * d
    det = a * d - b * c
    return np.sqrt(0.5 * (s + np.sqrt(np.maximum(s * s - 4 * det * det, 0.0))))


def image_position_bounds(O, model, grid, f, src_err, tris, pos, rtol):
    """Bound on |x_gpu - x_oracle| for an image both sides found in the same
    triangle, from the deflection tolerance |da| <= rtol * scale at each
    vertex (Z20) and the source error.  The barycentric image is the affine
    map of the source-plane triangle onto the image-plane one:
    x = v_a + E_v E_u^-1 (p - u_a), E_v = [v_b - v_a, v_c - v_a],
    E_u = [u_b - u_a, u_c - u_a], u = v - f alpha.  With every unlensed vertex
    moved by at most du (f rtol |scale| plus rounding), the source by at most
    src_err and p inside the triangle (barycentric weights lambda >= 0, sum 1),
    x' - x = E_v (E_u + dE)^-1 (dp - sum_k lambda_k du_k) exactly, so
      |x' - x| <= |E_v E_u^-1| d / (1 - |dE| |E_u^-1|),
    d = src_err + max du, |dE| <= 2 sqrt 2 max du (spectral norms).  Each
    side's rounding of the orientations (8 u L^2 each, L the longest
    source-plane edge) and of the quotient is added.  inf where the triangle
    is too thin for the bound (|dE| |E_u^-1| >= 1/2)."""
    n = len(tris)
    if n == 0:
        return np.zeros(0)
    ij = np.array([tri_vertices(t, grid) for t in tris])  # (n, 3, 2)
    vx, vy = grid_points(grid, ij[..., 0], ij[..., 1])
    val, mag = O.eval_points(model, vx.ravel(), vy.ravel())
    ax, ay = val[0].reshape(n, 3), val[1].reshape(n, 3)
    da = rtol * np.hypot(mag[0], mag[1]).reshape(n, 3)
    ux, uy = vx - f * ax, vy - f * ay
    du = (f * da + 4 * U * math.sqrt(2.0) * (np.hypot(vx, vy) + f * np.hypot(ax, ay))).max(axis=1)
    d = du + src_err
    # E_u = [[e1x, e2x], [e1y, e2y]], its inverse's norm and E_v E_u^-1
    e1x, e1y = ux[:, 1] - ux[:, 0], uy[:, 1] - uy[:, 0]
    e2x, e2y = ux[:, 2] - ux[:, 0], uy[:, 2] - uy[:, 0]
    det = e1x * e2y - e2x * e1y
    w1x, w1y = vx[:, 1] - vx[:, 0], vy[:, 1] - vy[:, 0]
    w2x, w2y = vx[:, 2] - vx[:, 0], vy[:, 2] - vy[:, 0]
    with np.errstate(divide="ignore", invalid="ignore"):
        i11, i12, i21, i22 = e2y / det, -e2x / det, -e1y / det, e1x / det
        kappa = _norm2(i11, i12, i21, i22)
        J = _norm2(w1x * i11 + w2x * i21, w1x * i12 + w2x * i22,
                   w1y * i11 + w2y * i21, w1y * i12 + w2y * i22)
        t = 2 * math.sqrt(2.0) * du * kappa
        b = np.where(t < 0.5, J * d / (1 - t), np.inf)
        L = np.hypot(ux[:, [1, 2, 0]] - ux, uy[:, [1, 2, 0]] - uy).max(axis=1)
        cx, cy = vx.mean(axis=1), vy.mean(axis=1)
        R = np.hypot(vx - cx[:, None], vy - cy[:, None]).max(axis=1)
        rnd = 2 * 48 * U * L * L * R / np.abs(det)
    return b + rnd + 16 * U * (np.hypot(pos[:, 0], pos[:, 1]) + R)


def assign(ix, iy, cx, cy):
    """The assignment rule of the image-plane chi^2 (each image to its nearest
    constraint, ties to the lower index; each constraint keeps its nearest
    image, ties to the earlier one).  Returns, per constraint, the index of
    its image or -1, and the near-tie margins: for each image the gap between
    its nearest and second-nearest constraint distance, for each constraint
    the gap between its nearest and second-nearest assigned image."""
    ix, iy, cx, cy = (np.asarray(v, dtype=np.float64) for v in (ix, iy, cx, cy))
    M = len(cx)
    keep = np.full(M, -1)
    gap_img = np.full(len(ix), np.inf)
    gap_con = np.full(M, np.inf)
    if len(ix) == 0:
        return keep, gap_img, gap_con
    d = np.hypot(ix[:, None] - cx[None, :], iy[:, None] - cy[None, :])  # (n, M)
    pick = np.argmin(d * d, axis=1)
    if M > 1:
        srt = np.sort(d, axis=1)
        gap_img = srt[:, 1] - srt[:, 0]
    for j in range(M):
        ks = np.nonzero(pick == j)[0]
        if len(ks) == 0:
            continue
        dj = d[ks, j]
        keep[j] = ks[np.argmin(dj * dj)]
        if len(ks) > 1:
            s2 = np.sort(dj)
            gap_con[j] = s2[1] - s2[0]
    return keep, gap_img, gap_con


def system_term(ix, iy, cx, cy, sig, penalty):
    """chi^2 term and missing count of one system under the assignment rule."""
    keep, _, _ = assign(ix, iy, cx, cy)
    term, miss = 0.0, 0
    for j, k in enumerate(keep):
        if k < 0:
            term += penalty
            miss += 1
        else:
            term += ((ix[k] - cx[j]) ** 2 + (iy[k] - cy[j]) ** 2) / sig[j] ** 2
    return term, miss


def compare_image_plane(O, fixed, free, free_off, cat, grid, got, ref, samples, m0, rtol,
                        penalty):
    """GPU image-plane results against the oracle's, sample by sample and
    system by system, under bounds derived from the deflection tolerance rtol
    (Z20) and the certified edge margin (Z21):
      * a system whose image count differs is excused only when its source
        lies within the deflection error bound of a triangle edge of the
        unlensed grid (oracle's edge margin against f rtol max scale + the
        source error); it is then left out of the position and chi^2 checks
        and counted;
      * a system whose assignment has a near tie (two distances closer than
        the position bounds allow to tell apart) is left out of the chi^2
        check and counted;
      * every other image must lie within its position bound of the
        oracle's, and the sample's chi^2 (with the excused systems' terms
        left out on both sides) within sum_j (2 |d_j| dx_j + dx_j^2)/sigma^2
        plus rounding.
    `got` holds the GPU arrays of all samples (nimg, img_xy, chi2, nmissing),
    `ref` the oracle's for samples m0.. (nimg, x, y, tri, chi2, nmiss).
    Returns a dict of counts and the largest observed/bound ratios."""
    off = np.asarray(cat["off"])
    nsys = len(off) - 1
    kmax_g = got["img_xy"].shape[2]
    st = dict(excused=0, near_tie=0, images=0, pos_ratio=0.0, pos_err=0.0, chi2_ratio=0.0,
              chi2_rel=0.0)
    for m in samples:
        s = m - m0
        model = {k: np.concatenate([fixed[k], free[k][free_off[m]:free_off[m + 1]]])
                 for k in fixed}
        bx, by, sabs = O.unlens(fixed, free, free_off, m, cat)
        sx, sy = O.sources(fixed, free, free_off, m, cat)
        serr = source_errors(bx, by, sabs, cat, rtol)
        chi2_g, chi2_o, bound = float(got["chi2"][m]), float(ref["chi2"][s]), 0.0
        miss_g, miss_o = int(got["nmissing"][m]), int(ref["nmiss"][s])
        model_grid = {}

        def near_edge(i):
            """Z21: the oracle's source of system i lies within the deflection
            error bound of a triangle edge of its unlensed grid."""
            if not model_grid:
                ax, ay = O.alpha_grid(model, grid)
                _, mag = O.lens_map(model, grid, 1.0)
                model_grid.update(ax=ax, ay=ay, scale=float(np.hypot(mag[0], mag[1]).max()))
            margin = O.edge_margin(model_grid["ax"], model_grid["ay"], grid, cat["f"][i],
                                   sx[i], sy[i])
            allow = cat["f"][i] * rtol * model_grid["scale"] + serr[i] + 64 * U * 100.0
            return margin <= allow, margin, allow

        for i in range(nsys):
            o0, o1 = off[i], off[i + 1]
            cx, cy, sig = cat["x"][o0:o1], cat["y"][o0:o1], cat["sig"][o0:o1]
            ng, no = int(got["nimg"][m, i]), int(ref["nimg"][s, i])
            kg, ko = min(ng, kmax_g), min(no, ref["x"].shape[2])
            gx, gy = got["img_xy"][m, i, :kg, 0], got["img_xy"][m, i, :kg, 1]
            ox, oy = ref["x"][s, i, :ko], ref["y"][s, i, :ko]
            excuse = ng != no
            if not excuse:
                k = min(kg, ko)
                pos = np.stack([ox[:k], oy[:k]], axis=1)
                pb = image_position_bounds(O, model, grid, cat["f"][i], serr[i],
                                           ref["tri"][s, i, :k], pos, rtol)
                err = np.hypot(gx[:k] - ox[:k], gy[:k] - oy[:k])
                excuse = not np.all(err <= pb)
            if excuse:
                ok, margin, allow = near_edge(i)
                assert ok, (m, i, ng, no, margin, allow)
                st["excused"] += 1
            else:
                st["images"] += int(k)
                if k:
                    st["pos_ratio"] = max(st["pos_ratio"], float(np.max(err / pb)))
                    st["pos_err"] = max(st["pos_err"], float(err.max()))
                keep, gap_img, gap_con = assign(ox[:k], oy[:k], cx, cy)
                tie = k > 0 and (np.any(gap_img <= 2 * pb) or any(
                    gap_con[j] <= 2 * pb.max() for j in range(len(cx)) if keep[j] >= 0))
                if not tie:
                    for j, kk in enumerate(keep):
                        if kk >= 0:
                            dj = math.hypot(ox[kk] - cx[j], oy[kk] - cy[j])
                            bound += (2 * dj * pb[kk] + pb[kk] ** 2) / sig[j] ** 2
                    continue
                st["near_tie"] += 1
            # left out of the chi^2 comparison on both sides
            tg, mg = system_term(gx, gy, cx, cy, sig, penalty)
            to, mo = O.assign_system(ox, oy, cx, cy, sig, penalty)
            chi2_g -= tg
            chi2_o -= to
            miss_g -= mg
            miss_o -= mo
        assert miss_g == miss_o, (m, miss_g, miss_o)
        bound += 8 * U * nsys * (abs(chi2_o) + 1.0)
        dc = abs(chi2_g - chi2_o)
        assert dc <= bound, (m, chi2_g, chi2_o, bound)
        st["chi2_ratio"] = max(st["chi2_ratio"], dc / bound)
        st["chi2_rel"] = max(st["chi2_rel"], dc / max(abs(chi2_o), 1.0))
    return st
