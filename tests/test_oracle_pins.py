"""Pins of the FP64 oracle against what mathematics fixes independently of it.

Each test ties one part of the oracle to a closed form, an invariant, an
independent numerical route or a brute-force check, chosen so that a dropped
term, a sign error, a swapped index or a transposed operand fails at least one.
None of these re-types the oracle's own formula.
"""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

RNG = np.random.default_rng(12345)


def pot(x0=0.0, y0=0.0, b0=10.0, eps=0.0, phi=0.0, a=0.0, s=math.inf):
    return [x0, y0, b0, eps, phi, a, s]


def rot(phi):
    c, s = math.cos(phi), math.sin(phi)
    return np.array([[c, -s], [s, c]])


# --------------------------------------------------------------------------
# Singular isothermal sphere (dPIE with rcore = 0, rcut = inf, eps = 0)
# --------------------------------------------------------------------------
def test_sis_deflection_is_einstein_radius(oracle):
    """|alpha| = b0 (the Einstein radius) everywhere but the centre, pointing
    away from the centre; H = b0/r^3 (y^2, -xy, x^2); kappa = b0/(2r)."""
    b0 = 7.3
    for _ in range(50):
        x0, y0 = RNG.uniform(-5, 5, 2)
        r = 10 ** RNG.uniform(-3, 3)
        t = RNG.uniform(0, 2 * math.pi)
        x, y = x0 + r * math.cos(t), y0 + r * math.sin(t)
        v, m = oracle.pot_eval(pot(x0, y0, b0), x, y)
        dx, dy = x - x0, y - y0
        rr = math.hypot(dx, dy)
        assert math.hypot(v[0], v[1]) == pytest.approx(b0, rel=1e-14)
        assert v[0] * dx + v[1] * dy > 0
        assert v[2] == pytest.approx(b0 * dy * dy / rr ** 3, rel=1e-12, abs=1e-14 * b0 / rr)
        assert v[3] == pytest.approx(-b0 * dx * dy / rr ** 3, rel=1e-12, abs=1e-14 * b0 / rr)
        assert v[4] == pytest.approx(b0 * dx * dx / rr ** 3, rel=1e-12, abs=1e-14 * b0 / rr)
        assert 0.5 * (v[2] + v[4]) == pytest.approx(b0 / (2 * rr), rel=1e-13)


def test_singular_centre_contributes_zero(oracle):
    v, m = oracle.pot_eval(pot(1.5, -2.0, 5.0, eps=0.3, a=0.0, s=20.0), 1.5, -2.0)
    assert np.all(v == 0) and np.all(m == 0)
    # a cored potential is regular at its centre: alpha = 0, H finite and positive
    v, _ = oracle.pot_eval(pot(1.5, -2.0, 5.0, eps=0.0, a=0.5, s=20.0), 1.5, -2.0)
    assert v[0] == 0 and v[1] == 0 and v[2] > 0 and v[2] == v[4] and v[3] == 0


# --------------------------------------------------------------------------
# Circular dPIE closed form
# --------------------------------------------------------------------------
@pytest.mark.parametrize("a,s", [(0.05, 10.0), (1.0, 30.0), (5.0, 1000.0), (0.0, 50.0)])
def test_circular_dpie_closed_form(oracle, a, s):
    """alpha(r) = b0 F [sqrt(a^2+r^2) - a - sqrt(s^2+r^2) + s]/r, F = s/(s-a),
    directed along the radius vector (enclosed-mass form of the circular dPIE)."""
    b0 = 12.0
    F = s / (s - a)
    for r in [1e-3, 0.07, 0.9, 3.0, 17.0, 120.0, 5000.0]:
        t = RNG.uniform(0, 2 * math.pi)
        x, y = r * math.cos(t), r * math.sin(t)
        v, m = oracle.pot_eval(pot(0, 0, b0, 0.0, RNG.uniform(0, 3), a, s), x, y)
        rr = math.hypot(x, y)
        with mp.workdps(50):
            mpr = mp.mpf(rr)
            ref = float(b0 * F * (mp.sqrt(a * a + mpr ** 2) - a - mp.sqrt(s * s + mpr ** 2) + s)
                        / mpr)
        assert math.hypot(v[0], v[1]) == pytest.approx(ref, rel=1e-12, abs=1e-15 * m[0])
        assert v[0] * x + v[1] * y > 0


# --------------------------------------------------------------------------
# Elliptical dPIE: convergence, FD consistency, independent quadrature
# --------------------------------------------------------------------------
def rand_pot(eps_max=0.5):
    return pot(RNG.uniform(-3, 3), RNG.uniform(-3, 3), RNG.uniform(0.5, 40),
               RNG.uniform(1e-3, eps_max), RNG.uniform(0, math.pi),
               RNG.uniform(0.01, 5), RNG.uniform(8, 500))


def dpie_kappa(p, x, y):
    """Surface density of the dPIE (Eliasdottir et al. 2007) in units of the
    critical density, with the Kassiola-Kovner elliptical radius."""
    x0, y0, b0, eps, phi, a, s = p
    c, sn = math.cos(phi), math.sin(phi)
    dx, dy = x - x0, y - y0
    xp, yp = dx * c + dy * sn, -dx * sn + dy * c
    rho2 = xp ** 2 / (1 + eps) ** 2 + yp ** 2 / (1 - eps) ** 2
    F = s / (s - a)
    return 0.5 * b0 * F * (1 / math.sqrt(a * a + rho2) - 1 / math.sqrt(s * s + rho2))


def test_elliptical_convergence_matches_surface_density(oracle):
    """kappa = (psi_xx + psi_yy)/2 (Poisson: the Laplacian of psi is twice kappa)."""
    for _ in range(200):
        p = rand_pot()
        x, y = RNG.uniform(-60, 60, 2) * 10 ** RNG.uniform(-2, 0)
        v, m = oracle.pot_eval(p, x, y)
        k = dpie_kappa(p, x, y)
        assert 0.5 * (v[2] + v[4]) == pytest.approx(k, abs=1e-13 * (m[2] + m[4]), rel=1e-12)


def test_hessian_is_derivative_of_deflection(oracle):
    """Central finite differences of alpha reproduce H (and d ax/dy = d ay/dx:
    alpha is a gradient), to the O(h^2) truncation of the difference."""
    for _ in range(60):
        p = rand_pot()
        x, y = RNG.uniform(-40, 40, 2)
        h = 1e-4
        ax_px, _ = oracle.pot_eval(p, x + h, y)
        ax_mx, _ = oracle.pot_eval(p, x - h, y)
        ay_py, _ = oracle.pot_eval(p, x, y + h)
        ay_my, _ = oracle.pot_eval(p, x, y - h)
        v, m = oracle.pot_eval(p, x, y)
        dxx = (ax_px[0] - ax_mx[0]) / (2 * h)
        dyx = (ax_px[1] - ax_mx[1]) / (2 * h)
        dxy = (ay_py[0] - ay_my[0]) / (2 * h)
        dyy = (ay_py[1] - ay_my[1]) / (2 * h)
        scale = max(m[2], m[3], m[4]) + 1e-300
        tol = 1e-6 * scale + 1e-9 * max(m[0], m[1])
        assert abs(dxx - v[2]) < tol
        assert abs(dyy - v[4]) < tol
        assert abs(dxy - v[3]) < tol
        assert abs(dyx - v[3]) < tol


def schramm_alpha(p, x, y):
    """Deflection of a homoeoidal lens by direct quadrature of its convergence
    (Schramm 1990; Keeton 2001 eqs. for kappa(xi^2), xi^2 = x^2 + y^2/q^2):
    ax = q x J0, ay = q y J1, J_n = int_0^1 kappa(xi(u)^2) / (1-(1-q^2)u)^(n+1/2) du,
    xi(u)^2 = u (x^2 + y^2/(1-(1-q^2)u)).  Evaluated in the potential's frame
    and rotated back with a numpy rotation matrix."""
    x0, y0, b0, eps, phi, a, s = p
    q = (1 - eps) / (1 + eps)
    R = rot(phi)
    xp, yp = R.T @ np.array([x - x0, y - y0])
    F = s / (s - a)

    def kap(xi2):
        rho2 = xi2 / (1 + eps) ** 2
        return 0.5 * b0 * F * (1 / math.sqrt(a * a + rho2) - 1 / math.sqrt(s * s + rho2))

    def J(n):
        f = lambda u: kap(u * (xp * xp + yp * yp / (1 - (1 - q * q) * u))) / (
            1 - (1 - q * q) * u) ** (n + 0.5)
        return integrate.quad(f, 0, 1, epsabs=0, epsrel=1e-13, limit=400)[0]

    return R @ np.array([q * xp * J(0), q * yp * J(1)])


def test_elliptical_deflection_by_independent_quadrature(oracle):
    """The oracle's closed form against a quadrature of the surface density.
    With div alpha = 2 kappa, curl alpha = 0 and decay, this fixes alpha."""
    for _ in range(40):
        p = rand_pot()
        p[5] = max(p[5], 0.05)
        x, y = p[0] + RNG.uniform(-50, 50), p[1] + RNG.uniform(-50, 50)
        v, m = oracle.pot_eval(p, x, y)
        ref = schramm_alpha(p, x, y)
        assert abs(v[0] - ref[0]) < 1e-11 * (m[0] + m[1])
        assert abs(v[1] - ref[1]) < 1e-11 * (m[0] + m[1])


def test_far_field_monopole(oracle):
    """|alpha| r -> (1 - eps^2) b0 s: the finite total mass of the dPIE (the
    elliptical radius scales areas by (1+eps)(1-eps))."""
    for _ in range(20):
        p = rand_pot()
        s = p[6]
        r = 1e6 * s
        t = RNG.uniform(0, 2 * math.pi)
        x, y = p[0] + r * math.cos(t), p[1] + r * math.sin(t)
        v, _ = oracle.pot_eval(p, x, y)
        assert math.hypot(v[0], v[1]) * r == pytest.approx((1 - p[3] ** 2) * p[2] * s, rel=1e-5)


@pytest.mark.parametrize("eps", [1e-12, 1e-8, 1e-4])
def test_small_ellipticity_is_continuous_with_circular(oracle, eps):
    for _ in range(20):
        p = rand_pot()
        p0 = list(p)
        p0[3] = 0.0
        p[3] = eps
        x, y = RNG.uniform(-30, 30, 2)
        v, m = oracle.pot_eval(p, x, y)
        v0, _ = oracle.pot_eval(p0, x, y)
        assert np.all(np.abs(v - v0) <= 10 * eps * m + 1e-15 * m)


def test_sis_is_the_limit_of_core_to_zero_and_cut_to_infinity(oracle):
    x, y = 3.0, -4.0
    v_sis, _ = oracle.pot_eval(pot(0, 0, 10.0), x, y)
    v_lim, _ = oracle.pot_eval(pot(0, 0, 10.0, 0.0, 0.0, 1e-9, 1e9), x, y)
    assert np.allclose(v_lim, v_sis, rtol=1e-8, atol=1e-8)


def test_rotation_covariance(oracle):
    """Rotating the potential about its centre and the point with it maps
    alpha -> R alpha and H -> R H R^T."""
    for _ in range(30):
        p = rand_pot()
        x, y = p[0] + RNG.uniform(-30, 30), p[1] + RNG.uniform(-30, 30)
        t = RNG.uniform(0, 2 * math.pi)
        R = rot(t)
        q = dict(enumerate(p))
        p2 = list(p)
        p2[4] = p[4] + t
        xr, yr = np.array([p[0], p[1]]) + R @ np.array([x - p[0], y - p[1]])
        v, m = oracle.pot_eval(p, x, y)
        v2, _ = oracle.pot_eval(p2, xr, yr)
        a1 = R @ v[:2]
        H = np.array([[v[2], v[3]], [v[3], v[4]]])
        H1 = R @ H @ R.T
        sc = m.max()
        assert np.allclose(v2[:2], a1, atol=1e-12 * sc, rtol=0)
        assert np.allclose([v2[2], v2[3], v2[4]], [H1[0, 0], H1[0, 1], H1[1, 1]],
                           atol=1e-12 * sc, rtol=0)


def test_superposition_and_permutation(oracle):
    n = 12
    P = {k: [] for k in ("x0", "y0", "b0", "eps", "phi", "rcore", "rcut")}
    for _ in range(n):
        for k, v in zip(P, rand_pot()):
            P[k].append(v)
    P = {k: np.array(v) for k, v in P.items()}
    grid = (7, 5, -20.0, -15.0, 6.1, 7.3)
    full, mag = oracle.lens_map(P, grid, 0.7)
    A = {k: v[:5] for k, v in P.items()}
    B = {k: v[5:] for k, v in P.items()}
    perm = RNG.permutation(n)
    Pp = {k: v[perm] for k, v in P.items()}
    a, _ = oracle.lens_map(A, grid, 0.7)
    b, _ = oracle.lens_map(B, grid, 0.7)
    pp, _ = oracle.lens_map(Pp, grid, 0.7)
    assert np.all(np.abs(a + b - full) <= 1e-14 * mag)
    assert np.all(np.abs(pp - full) <= 1e-14 * mag)
    # each pixel of the map is the single-point sum times Dls/Ds
    j, i = 3, 4
    v, _ = oracle.eval_points(P, [grid[2] + i * grid[4]], [grid[3] + j * grid[5]])
    assert np.allclose(full[:, j, i], 0.7 * v[:, 0], rtol=0, atol=1e-15 * mag[:, j, i].max())


def test_closed_form_rounding_against_40_digit_evaluation(oracle):
    """The oracle's own rounding: the same dPIE evaluated with 40-digit
    arithmetic; the FP64 result must sit within a few 1e-16 of the scale."""
    def core(b0, eps, w, xp, yp):
        b0, eps, w, xp, yp = map(mp.mpf, (b0, eps, w, xp, yp))
        q = (1 - eps) / (1 + eps)
        S = (1 + eps) * w
        psi = mp.sqrt(q * q * (S * S + xp * xp) + yp * yp)
        k = mp.sqrt(1 - q * q)
        b = b0 * (1 + eps)  # Keeton's amplitude
        ax = b * q / k * mp.atan(k * xp / (psi + S))
        ay = b * q / k * mp.atanh(k * yp / (psi + q * q * S))
        D = (1 + q * q) * S * S + 2 * psi * S + xp * xp + yp * yp
        h = b * q / psi
        return [ax, ay, h * (q * q * S * S + yp * yp + S * psi) / D, -h * xp * yp / D,
                h * (S * S + xp * xp + S * psi) / D]

    for _ in range(40):
        with mp.workdps(40):
            _check_one_40_digit(oracle, core)


def _check_one_40_digit(oracle, core):
    if True:
        p = rand_pot()
        x, y = RNG.uniform(-50, 50, 2)
        x0, y0, b0, eps, phi, a, s = map(mp.mpf, p)
        c, sn = mp.cos(phi), mp.sin(phi)
        dx, dy = mp.mpf(x) - x0, mp.mpf(y) - y0
        xp, yp = dx * c + dy * sn, -dx * sn + dy * c
        A, Sx = core(b0, eps, a, xp, yp), core(b0, eps, s, xp, yp)
        F = s / (s - a)
        d = [F * (u - w) for u, w in zip(A, Sx)]
        ref = [c * d[0] - sn * d[1], sn * d[0] + c * d[1],
               c * c * d[2] - 2 * c * sn * d[3] + sn * sn * d[4],
               c * sn * (d[2] - d[4]) + (c * c - sn * sn) * d[3],
               sn * sn * d[2] + 2 * c * sn * d[3] + c * c * d[4]]
        v, m = oracle.pot_eval(p, x, y)
        for ch in range(5):
            assert abs(v[ch] - float(ref[ch])) <= 2e-15 * m[ch] + 1e-300


# --------------------------------------------------------------------------
# Physical parameters and distances
# --------------------------------------------------------------------------
def test_parameter_conversions(oracle):
    # e = (a^2 - b^2)/(a^2 + b^2) and eps = (a - b)/(a + b) for axes a = 1+eps, b = 1-eps
    for eps in [0.0, 1e-9, 0.01, 0.153536, 0.3, 0.8]:
        e = 2 * eps / (1 + eps * eps)
        assert oracle.eps_from_e([e])[0] == pytest.approx(eps, rel=1e-12, abs=1e-300)
    # sigma = 1000 km/s, 6 pi (sigma/c)^2 rad in arcsec
    want = 6 * math.pi * (1000 / 299792.458) ** 2 * 206264.80624709636
    assert oracle.b0_from_sigma([1000.0])[0] == pytest.approx(want, rel=1e-14)
    assert oracle.b0_from_sigma([1000.0], 1)[0] == pytest.approx(want * 4 / 6, rel=1e-14)


def test_distance_ratio_einstein_de_sitter(oracle):
    """Omega_m = 1: chi(z) = 2 (1 - 1/sqrt(1+z)) in units of c/H0."""
    chi = lambda z: 2 * (1 - 1 / math.sqrt(1 + z))
    for zl, zs in [(0.1, 0.5), (0.4, 2.0), (0.3, 6.0), (1.0, 1.0001)]:
        assert oracle.dlsds(zl, zs, 1.0, 0.0) == pytest.approx(1 - chi(zl) / chi(zs), rel=1e-10)


def test_distance_ratio_flat_lcdm_by_quadrature(oracle):
    E = lambda z: 1 / math.sqrt(0.3 * (1 + z) ** 3 + 0.7)
    chi = lambda z: integrate.quad(E, 0, z, epsabs=0, epsrel=1e-13)[0]
    for zl, zs in [(0.4, 1.0), (0.4, 2.0), (0.4, 6.0), (0.2, 0.25)]:
        assert oracle.dlsds(zl, zs) == pytest.approx(1 - chi(zl) / chi(zs), rel=1e-11)
    with pytest.raises(ValueError):
        oracle.dlsds(2.0, 1.0)
    with pytest.raises(ValueError):
        oracle.dlsds(0.4, 2.0, 0.3, 0.6)


# --------------------------------------------------------------------------
# Exact orientation predicate (brute force with exact rationals)
# --------------------------------------------------------------------------
def frac_orient(a, b, p):
    ax, ay, bx, by, px, py = map(Fraction, (*a, *b, *p))
    d = (bx - ax) * (py - ay) - (by - ay) * (px - ax)
    return (d > 0) - (d < 0)


def test_orientation_sign_is_exact(oracle):
    cases = []
    for _ in range(3000):
        cases.append(tuple(RNG.uniform(-100, 100, 6)))
    # points exactly on a line through two representable points
    for _ in range(2000):
        ax, ay = RNG.uniform(-50, 50, 2)
        dx, dy = RNG.uniform(-1, 1, 2)
        t1, t2 = RNG.integers(-64, 64, 2) / 64.0
        cases.append((ax, ay, ax + t1 * dx, ay + t1 * dy, ax + t2 * dx, ay + t2 * dy))
    # nearly collinear: nudge by a few ulp
    for _ in range(2000):
        ax, ay, bx, by = RNG.uniform(-1, 1, 4) * 10 ** RNG.uniform(-3, 2)
        t = RNG.uniform(-2, 3)
        px, py = ax + t * (bx - ax), ay + t * (by - ay)
        px = np.nextafter(px, px + RNG.choice([-1, 1]) * 1e300 * int(RNG.integers(0, 2)))
        cases.append((ax, ay, bx, by, px, py))
    # tiny and huge magnitudes
    for _ in range(500):
        s = 10 ** RNG.uniform(-200, 200)
        cases.append(tuple(RNG.uniform(-1, 1, 6) * s))
    cases.append((0.0, 0.0, 0.0, 0.0, 1.0, 1.0))
    cases.append((5e-324, 0.0, 0.0, 5e-324, 5e-324, 5e-324))
    for c in cases:
        c = tuple(float(v) for v in c)
        assert oracle.orient_exact(*c) == frac_orient(c[0:2], c[2:4], c[4:6]), c


def test_perturbed_orientation_tie_rule(oracle):
    # p on the edge a->b: the decision falls to -(by-ay), then (bx-ax)
    assert oracle.orient_perturbed(0, 0, 0, 1, 0, 0.5) == -1   # upward edge: p+d is right
    assert oracle.orient_perturbed(0, 1, 0, 0, 0, 0.5) == 1
    assert oracle.orient_perturbed(0, 0, 1, 0, 0.5, 0) == 1    # horizontal: p+(d, d^2) is above
    assert oracle.orient_perturbed(1, 0, 0, 0, 0.5, 0) == -1
    assert oracle.orient_perturbed(0, 0, 0, 0, 0.5, 0) == 0


# --------------------------------------------------------------------------
# Brute-force image search
# --------------------------------------------------------------------------
def test_zero_lens_gives_one_image_at_the_source(oracle):
    grid = (41, 37, -10.0, -9.0, 0.5, 0.5)
    ax = np.zeros((37, 41))
    for _ in range(200):
        px, py = RNG.uniform(-9.9, 9.9), RNG.uniform(-8.9, 8.9)
        n, tri, ix, iy = oracle.find_images(ax, ax, grid, 0.8, px, py)
        assert n == 1
        assert ix[0] == pytest.approx(px, abs=1e-13) and iy[0] == pytest.approx(py, abs=1e-13)
    # a source exactly on grid vertices and edges still lands in exactly one triangle
    for i, j in [(3, 4), (10, 10), (20, 30)]:
        px, py = grid[2] + i * grid[4], grid[3] + j * grid[5]
        for qx, qy in [(px, py), (px + 0.25, py), (px, py + 0.25), (px + 0.25, py + 0.25)]:
            n, tri, ix, iy = oracle.find_images(ax, ax, grid, 1.0, qx, qy)
            assert n == 1
    # outside the grid: none
    assert oracle.find_images(ax, ax, grid, 1.0, 50.0, 0.0)[0] == 0


def radial_images(b0, a, beta):
    """Images of a source at radius beta for a circular cored isothermal lens
    (rcut = inf): roots of r - alpha(r) = beta along the source direction,
    alpha(r) = b0 (sqrt(a^2 + r^2) - a)/r, found by bisection."""
    alpha = lambda r: b0 * (math.sqrt(a * a + r * r) - a) / r if r != 0 else 0.0
    g = lambda r: r - alpha(r) - beta
    roots, xs = [], np.linspace(-60, 60, 24001)
    for lo, hi in zip(xs[:-1], xs[1:]):
        if g(lo) == 0:
            roots.append(lo)
        elif g(lo) * g(hi) < 0:
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if g(lo) * g(mid) <= 0:
                    hi = mid
                else:
                    lo = mid
            roots.append(0.5 * (lo + hi))
    return roots


def test_cored_isothermal_images_and_odd_multiplicity(oracle):
    """Non-singular circular lens: 3 images inside the caustic, 1 outside (odd
    number theorem), at the roots of the radial lens equation up to the grid's
    linear-interpolation error."""
    b0, a = 10.0, 1.0
    grid = (451, 451, -45.0, -45.0, 0.2, 0.2)
    n = grid[0]
    xs = grid[2] + np.arange(n) * grid[4]
    X, Y = np.meshgrid(xs, xs)
    pots = dict(x0=[0.3], y0=[-0.2], b0=[b0], eps=[0.0], phi=[0.0], rcore=[a], rcut=[np.inf])
    axg, ayg = oracle.alpha_grid(pots, grid)
    for beta_r, want in [(0.5, 3), (2.0, 3), (15.0, 1), (25.0, 1)]:
        t = RNG.uniform(0, 2 * math.pi)
        px, py = 0.3 + beta_r * math.cos(t), -0.2 + beta_r * math.sin(t)
        cnt, tri, ix, iy = oracle.find_images(axg, ayg, grid, 1.0, px, py)
        assert cnt == want
        roots = radial_images(b0, a, beta_r)
        assert len(roots) == want
        got = sorted(((x - 0.3) * math.cos(t) + (y + 0.2) * math.sin(t)) for x, y in zip(ix, iy))
        for g, r in zip(got, sorted(roots)):
            assert abs(g - r) < 0.05


def grid_edge_distance(grid, px, py):
    """Distance from (px, py) to the nearest triangle edge of an unlensed grid
    split into T0/T1 by the anti-diagonal of each cell, in closed form: inside
    the grid's rectangle the nearest edge is one of the containing cell's four
    sides or its anti-diagonal u + v = 1 (local coordinates u, v in [0, 1]);
    outside it, the rectangle's boundary is made of edges, so the distance is
    the distance to the rectangle."""
    nx, ny, x0, y0, dx, dy = grid
    X1, Y1 = x0 + (nx - 1) * dx, y0 + (ny - 1) * dy
    ox = max(x0 - px, 0.0, px - X1)
    oy = max(y0 - py, 0.0, py - Y1)
    if ox > 0 or oy > 0:
        return math.hypot(ox, oy)
    i = min(max(int(math.floor((px - x0) / dx)), 0), nx - 2)
    j = min(max(int(math.floor((py - y0) / dy)), 0), ny - 2)
    u, v = (px - (x0 + i * dx)) / dx, (py - (y0 + j * dy)) / dy
    diag = abs(u + v - 1.0) * dx * dy / math.hypot(dx, dy)
    return min(u * dx, (1 - u) * dx, v * dy, (1 - v) * dy, diag)


def test_edge_margin_closed_forms(oracle):
    """The margin of a source to the nearest triangle edge of the unlensed
    grid (the certificate that excuses a multiplicity difference between two
    evaluations): with no lens the closed form above, at random points, on
    vertices, grid lines and anti-diagonals (margin 0), past the last column
    and row and past the corners; with a uniform deflection c the grid is
    translated by -f c; with a mass sheet alpha = (k1 x, k2 y) it is rescaled
    by (1 - f k1, 1 - f k2), which exercises the per-vertex deflection."""
    grid = (13, 11, -3.0, -2.5, 0.5, 0.4)
    nx, ny, x0, y0, dx, dy = grid
    X1, Y1 = x0 + (nx - 1) * dx, y0 + (ny - 1) * dy
    zero = np.zeros((ny, nx))
    pts = [(RNG.uniform(x0 - 1, X1 + 1), RNG.uniform(y0 - 1, Y1 + 1)) for _ in range(300)]
    pts += [(x0 + 3 * dx, y0 + 4 * dy), (x0 + 5.5 * dx, y0 + 2 * dy), (x0 + 7 * dx, y0 + 0.3 * dy),
            (x0 + 4.25 * dx, y0 + 6.75 * dy),    # on an anti-diagonal
            (x0 + 2.2 * dx, y0 + 0.75 * dy),     # nearest edge: the anti-diagonal
            (X1 + 0.3, y0 + 4.5 * dy), (x0 + 6.5 * dx, Y1 + 0.2), (X1 + 0.3, Y1 + 0.4),
            (x0 - 0.2, y0 - 0.1), (X1 - 0.05, y0 + 5.5 * dy), (x0 + 6.5 * dx, Y1 - 0.03)]
    for px, py in pts:
        want = grid_edge_distance(grid, px, py)
        got = oracle.edge_margin(zero, zero, grid, 0.7, px, py)
        assert got == pytest.approx(want, abs=1e-12), (px, py, got, want)
    # a uniform deflection: the unlensed grid is the grid moved by -f c
    f, cx, cy = 0.6, 1.7, -0.9
    for px, py in pts[:120]:
        want = grid_edge_distance(grid, px + f * cx, py + f * cy)
        got = oracle.edge_margin(zero + cx, zero + cy, grid, f, px, py)
        assert got == pytest.approx(want, abs=1e-12)
    # an anisotropic mass sheet: unlensed vertex (1 - f k1) x, (1 - f k2) y
    k1, k2 = 0.35, -0.2
    xs, ys = x0 + np.arange(nx) * dx, y0 + np.arange(ny) * dy
    X, Y = np.meshgrid(xs, ys)
    sx, sy = 1 - f * k1, 1 - f * k2
    sheet = (nx, ny, x0 * sx, y0 * sy, dx * sx, dy * sy)
    for px, py in pts[:120] + pts[300:]:
        want = grid_edge_distance(sheet, px, py)
        got = oracle.edge_margin(k1 * X, k2 * Y, grid, f, px, py)
        assert got == pytest.approx(want, abs=1e-12)


def test_assignment_rules(oracle):
    cx, cy, sig = [0.0, 1.0, 5.0], [0.0, 0.0, 0.0], [0.5, 0.5, 1.0]
    # image 0 nearest constraint 0, image 1 nearest constraint 1, none for 2
    part, miss = oracle.assign_system([0.1, 1.2], [0.0, 0.0], cx, cy, sig, 7.0)
    assert miss == 1
    assert part == pytest.approx(0.01 / 0.25 + 0.04 / 0.25 + 7.0)
    # two images pick constraint 0: the nearer is kept; an exact tie keeps the first
    part, miss = oracle.assign_system([0.3, -0.2, 0.2], [0.0, 0.0, 0.0], cx, cy, sig, 0.0)
    assert miss == 2 and part == pytest.approx(0.04 / 0.25)
    # an image equidistant from two constraints goes to the lower index
    part, miss = oracle.assign_system([0.5], [0.0], cx, cy, sig, 0.0)
    assert miss == 2 and part == pytest.approx(0.25 / 0.25)


# --------------------------------------------------------------------------
# chi^2
# --------------------------------------------------------------------------
def empty_pots():
    return {k: np.zeros(0) for k in ("x0", "y0", "b0", "eps", "phi", "rcore", "rcut")}


def small_catalog(rng, nsys=5):
    off, x, y, sig = [0], [], [], []
    for i in range(nsys):
        m = int(rng.integers(1, 5))
        x += list(rng.uniform(-20, 20, m))
        y += list(rng.uniform(-20, 20, m))
        sig += list(rng.uniform(0.03, 0.1, m))
        off.append(len(x))
    return dict(off=np.array(off, np.int32), x=np.array(x), y=np.array(y),
                sig=np.array(sig), f=rng.uniform(0.5, 0.8, nsys))


def test_source_chi2_zero_lens_closed_form(oracle):
    cat = small_catalog(np.random.default_rng(3))
    chi2 = oracle.chi2_source(empty_pots(), empty_pots(), np.zeros(4, np.int32), cat)
    want = 0.0
    for i in range(len(cat["off"]) - 1):
        s = slice(cat["off"][i], cat["off"][i + 1])
        x, y, sg = cat["x"][s], cat["y"][s], cat["sig"][s]
        want += np.sum(((x - x.mean()) ** 2 + (y - y.mean()) ** 2) / sg ** 2)
    assert np.allclose(chi2, want, rtol=1e-13)


def test_source_chi2_invariant_under_translation_and_rotation(oracle):
    rng = np.random.default_rng(9)
    cat = small_catalog(rng)
    P = {k: [] for k in ("x0", "y0", "b0", "eps", "phi", "rcore", "rcut")}
    for _ in range(4):
        for k, v in zip(P, rand_pot()):
            P[k].append(v)
    P = {k: np.array(v) for k, v in P.items()}
    off = np.array([0, 2, 4], np.int32)
    fixed = {k: v[:0] for k, v in P.items()}
    base = oracle.chi2_source(fixed, P, off, cat)
    t = 0.7
    R = rot(t)
    shift = np.array([3.0, -1.5])
    P2 = dict(P)
    c2 = R @ np.stack([P["x0"], P["y0"]]) + shift[:, None]
    P2["x0"], P2["y0"], P2["phi"] = c2[0], c2[1], P["phi"] + t
    cat2 = dict(cat)
    cc = R @ np.stack([cat["x"], cat["y"]]) + shift[:, None]
    cat2["x"], cat2["y"] = cc[0], cc[1]
    moved = oracle.chi2_source(fixed, P2, off, cat2)
    assert np.allclose(moved, base, rtol=1e-9)


def test_source_chi2_vanishes_for_noise_free_constraints_of_the_true_model(oracle):
    """The stored catalogue's noise-free positions are exact images of the true
    config-3 model, so every system unlenses to one point: chi^2 ~ 0."""
    from paper_2004_06352_amd import inputs
    cat = oracle.catalog_f(inputs.load_catalog(), inputs.ZL)
    cat0 = dict(cat, x=cat["x_true"], y=cat["y_true"])
    fixed = oracle.phys_to_pots(inputs.fixed_galaxies(3))
    free = oracle.phys_to_pots(inputs.truth_free())
    off = np.array([0, inputs.N_FREE], np.int32)
    chi0 = oracle.chi2_source(fixed, free, off, cat0)[0]
    assert chi0 < 1e-12
    # with the 0.05" noise the source-plane scatter is of order the image count
    # scaled by the squared magnifications' inverse: clearly nonzero
    assert oracle.chi2_source(fixed, free, off, cat)[0] > 1.0


def test_image_chi2_zero_lens_closed_form(oracle):
    """No lens: each system's source is the mean of its constraints, found once
    at that point; the nearest constraint takes it, the others are missing."""
    cat = small_catalog(np.random.default_rng(5), nsys=6)
    grid = (101, 101, -25.0, -25.0, 0.5, 0.5)
    pen = 3.0
    res = oracle.chi2_image(empty_pots(), empty_pots(), np.zeros(2, np.int32), cat, grid,
                            kmax=4, penalty=pen)
    want, miss = 0.0, 0
    for i in range(len(cat["off"]) - 1):
        s = slice(cat["off"][i], cat["off"][i + 1])
        x, y, sg = cat["x"][s], cat["y"][s], cat["sig"][s]
        mx, my = x.mean(), y.mean()
        d2 = (x - mx) ** 2 + (y - my) ** 2
        j = int(np.argmin(d2))
        want += d2[j] / sg[j] ** 2 + pen * (len(x) - 1)
        miss += len(x) - 1
        assert res["nimg"][0, i] == 1
        assert res["x"][0, i, 0] == pytest.approx(mx, abs=1e-12)
        assert res["y"][0, i, 0] == pytest.approx(my, abs=1e-12)
    assert res["chi2"][0] == pytest.approx(want, rel=1e-9)
    assert res["nmiss"][0] == miss


# --------------------------------------------------------------------------
# Derived maps: convergence, shear, det of the inverse magnification matrix, mu
# --------------------------------------------------------------------------
def _derived_at(oracle, p, x, y, f=1.0):
    v, m = oracle.pot_eval(p, x, y)
    d = oracle.derived(np.array([f * v[2]]), np.array([f * v[3]]), np.array([f * v[4]]))
    return {k: float(val[0]) for k, val in d.items()}, v, m


def test_derived_sis_closed_form(oracle):
    """Singular isothermal sphere scaled by f = Dls/Ds: kappa = gamma = f b0/(2r),
    so det A^-1 = (1 - kappa)^2 - gamma^2 = 1 - f b0/r and mu = 1/(1 - f b0/r)
    (infinite on the Einstein ring r = f b0, negative inside it)."""
    b0 = 9.0
    for _ in range(60):
        f = RNG.uniform(0.3, 1.0)
        r = 10 ** RNG.uniform(-1, 2.5)
        t = RNG.uniform(0, 2 * math.pi)
        d, _, _ = _derived_at(oracle, pot(0, 0, b0), r * math.cos(t), r * math.sin(t), f)
        k = f * b0 / (2 * r)
        assert d["kappa"] == pytest.approx(k, rel=1e-13)
        assert d["gamma"] == pytest.approx(k, rel=1e-12)
        assert d["det"] == pytest.approx(1 - f * b0 / r, rel=1e-10, abs=1e-13 * (1 + f * b0 / r))
        if abs(1 - f * b0 / r) > 1e-3:
            assert d["mu"] == pytest.approx(1 / (1 - f * b0 / r), rel=1e-9)
        # tangential shear: gamma1 + i gamma2 = -gamma e^{2 i t} for a point mass-like profile
        assert d["gamma1"] == pytest.approx(-k * math.cos(2 * t), abs=1e-12 * k)
        assert d["gamma2"] == pytest.approx(-k * math.sin(2 * t), abs=1e-12 * k)


@pytest.mark.parametrize("a,s", [(0.5, 30.0), (2.0, 400.0)])
def test_derived_circular_dpie_shear_is_mean_minus_local_convergence(oracle, a, s):
    """For an axisymmetric lens gamma(r) = kbar(r) - kappa(r), with the mean
    convergence kbar = alpha(r)/r from the enclosed-mass deflection and
    kappa(r) = (b0 F/2)[1/sqrt(a^2+r^2) - 1/sqrt(s^2+r^2)]."""
    b0 = 15.0
    F = s / (s - a)
    for r in [0.05, 0.8, 2.5, 11.0, 60.0, 900.0]:
        t = RNG.uniform(0, 2 * math.pi)
        d, _, m = _derived_at(oracle, pot(0, 0, b0, 0.0, RNG.uniform(0, 3), a, s),
                              r * math.cos(t), r * math.sin(t))
        with mp.workdps(50):
            R = mp.mpf(r)
            alpha = b0 * F * (mp.sqrt(a * a + R * R) - a - mp.sqrt(s * s + R * R) + s) / R
            kap = b0 * F / 2 * (1 / mp.sqrt(a * a + R * R) - 1 / mp.sqrt(s * s + R * R))
            gam = float(alpha / R - kap)
            kap = float(kap)
        scale = max(m[2], m[4]) + 1e-300
        assert d["kappa"] == pytest.approx(kap, rel=1e-12, abs=1e-14 * scale)
        assert d["gamma"] == pytest.approx(gam, rel=1e-9, abs=1e-13 * scale)


def test_derived_det_is_jacobian_of_lens_mapping(oracle):
    """det A^-1 equals the determinant of d beta / d theta for beta = theta - f alpha,
    by central differences of the deflection (O(h^2)); mu det = 1."""
    for _ in range(40):
        p = [RNG.uniform(-3, 3), RNG.uniform(-3, 3), RNG.uniform(2, 30), RNG.uniform(0, 0.5),
             RNG.uniform(0, math.pi), RNG.uniform(0.05, 4), RNG.uniform(20, 500)]
        f = RNG.uniform(0.4, 1.0)
        x, y = RNG.uniform(-40, 40, 2)
        h = 1e-4
        axp, _ = oracle.pot_eval(p, x + h, y)
        axm, _ = oracle.pot_eval(p, x - h, y)
        ayp, _ = oracle.pot_eval(p, x, y + h)
        aym, _ = oracle.pot_eval(p, x, y - h)
        j11 = 1 - f * (axp[0] - axm[0]) / (2 * h)
        j12 = -f * (ayp[0] - aym[0]) / (2 * h)
        j21 = -f * (axp[1] - axm[1]) / (2 * h)
        j22 = 1 - f * (ayp[1] - aym[1]) / (2 * h)
        d, v, m = _derived_at(oracle, p, x, y, f)
        scale = 1 + f * max(m[2], m[3], m[4])
        assert abs(d["det"] - (j11 * j22 - j12 * j21)) < 1e-6 * scale * scale
        assert d["mu"] * d["det"] == pytest.approx(1.0, rel=1e-14)


def test_derived_rotation_covariance(oracle):
    """Rotating lens and point by t leaves kappa, gamma, det unchanged and turns
    (gamma1, gamma2) by 2t."""
    for _ in range(30):
        p = [0.0, 0.0, RNG.uniform(2, 30), RNG.uniform(0, 0.5), RNG.uniform(0, math.pi),
             RNG.uniform(0.05, 4), RNG.uniform(20, 500)]
        x, y = RNG.uniform(-30, 30, 2)
        t = RNG.uniform(0, 2 * math.pi)
        q = list(p)
        q[4] = p[4] + t
        xr, yr = rot(t) @ np.array([x, y])
        d0, _, m = _derived_at(oracle, p, x, y)
        d1, _, _ = _derived_at(oracle, q, xr, yr)
        sc = max(m[2], m[3], m[4])
        for k in ("kappa", "gamma", "det"):
            assert d1[k] == pytest.approx(d0[k], rel=1e-11, abs=1e-12 * sc)
        g1 = d0["gamma1"] * math.cos(2 * t) - d0["gamma2"] * math.sin(2 * t)
        g2 = d0["gamma1"] * math.sin(2 * t) + d0["gamma2"] * math.cos(2 * t)
        assert d1["gamma1"] == pytest.approx(g1, abs=1e-11 * sc)
        assert d1["gamma2"] == pytest.approx(g2, abs=1e-11 * sc)


# --------------------------------------------------------------------------
# Image refinement (Newton on the lens equation)
# --------------------------------------------------------------------------
def test_refine_sis_images_are_exact(oracle):
    """SIS scaled by f: a source at beta has images at beta_hat (|beta| + f b0)
    and, when |beta| < f b0, at beta_hat (|beta| - f b0) on the other side.
    The start is within a fifth of the image's distance from the centre (at
    most 0.1"): Newton's method starts on the image's side of the singular
    centre, where the deflection is smooth."""
    rng = np.random.default_rng(7061)  # its own stream: independent of test order
    for _ in range(40):
        b0, f = rng.uniform(3, 30), rng.uniform(0.4, 1.0)
        x0, y0 = rng.uniform(-5, 5, 2)
        lens = dict(x0=[x0], y0=[y0], b0=[b0], eps=[0.0], phi=[0.0], rcore=[0.0], rcut=[math.inf])
        r = rng.uniform(0.05, 0.95) * f * b0
        t = rng.uniform(0, 2 * math.pi)
        beta = (x0 + r * math.cos(t), y0 + r * math.sin(t))
        for rad in (r + f * b0, r - f * b0):
            want = (x0 + rad * math.cos(t), y0 + rad * math.sin(t))
            d = min(0.1, 0.2 * abs(rad)) / math.sqrt(2.0)
            start = (want[0] + rng.uniform(-d, d), want[1] + rng.uniform(-d, d))
            x, y, it = oracle.refine_image(empty_pots(), lens, f, beta, start)
            assert it > 0
            assert math.hypot(x - want[0], y - want[1]) < 1e-12 * (1 + f * b0)


def test_refine_cored_lens_matches_radial_roots(oracle):
    """Circular cored isothermal lens: refined images sit on the roots of the
    radial lens equation (bisection to machine precision)."""
    b0, a = 10.0, 1.0
    lens = dict(x0=[0.3], y0=[-0.2], b0=[b0], eps=[0.0], phi=[0.0], rcore=[a], rcut=[math.inf])
    for beta_r in (0.5, 2.0, 15.0):
        t = RNG.uniform(0, 2 * math.pi)
        beta = (0.3 + beta_r * math.cos(t), -0.2 + beta_r * math.sin(t))
        for root in radial_images(b0, a, beta_r):
            start = (0.3 + (root + 0.05) * math.cos(t), -0.2 + (root + 0.05) * math.sin(t))
            x, y, it = oracle.refine_image(empty_pots(), lens, 1.0, beta, start)
            assert it > 0
            got = (x - 0.3) * math.cos(t) + (y + 0.2) * math.sin(t)
            assert abs(got - root) < 1e-9


def test_refine_failure_keeps_the_grid_estimate(oracle):
    lens = dict(x0=[0.0], y0=[0.0], b0=[10.0], eps=[0.2], phi=[0.3], rcore=[1.0], rcut=[500.0])
    x, y, it = oracle.refine_image(empty_pots(), lens, 1.0, (1.0, 0.5), (30.0, -20.0),
                                   max_iter=1, max_shift=0.5)
    assert it == -1 and (x, y) == (30.0, -20.0)


def test_refined_image_chi2_vanishes_for_noise_free_constraints(oracle):
    """The true model with its noise-free constraints: with refinement every
    predicted image lands on its constraint (chi^2 ~ 0); without it the grid's
    linear interpolation leaves a clearly nonzero chi^2."""
    from paper_2004_06352_amd import inputs
    cat = oracle.catalog_f(inputs.load_catalog(), inputs.ZL)
    cat0 = dict(cat, x=cat["x_true"], y=cat["y_true"])
    fixed = oracle.phys_to_pots(inputs.fixed_galaxies(3))
    free = oracle.phys_to_pots(inputs.truth_free())
    off = np.array([0, inputs.N_FREE], np.int32)
    grid = inputs.pixel_centre_grid(500, -75.0, 75.0)
    shift = 2 * max(grid[4], grid[5])
    plain = oracle.chi2_image(fixed, free, off, cat0, grid, kmax=16, penalty=100.0)
    ref = oracle.chi2_image(fixed, free, off, cat0, grid, kmax=16, penalty=100.0,
                            refine=(20, 1e-10, shift))
    assert plain["nmiss"][0] == ref["nmiss"][0] == 0 and ref["nfail"][0] == 0
    assert ref["chi2"][0] < 1e-10
    assert plain["chi2"][0] > 1e-4


# --------------------------------------------------------------------------
# Lensing potential and time-delay surface
# --------------------------------------------------------------------------
def test_potential_sis_is_b0_r(oracle):
    for _ in range(40):
        b0 = RNG.uniform(1, 40)
        x0, y0 = RNG.uniform(-5, 5, 2)
        r = 10 ** RNG.uniform(-3, 3)
        t = RNG.uniform(0, 2 * math.pi)
        v, m = oracle.potential_eval(pot(x0, y0, b0), x0 + r * math.cos(t), y0 + r * math.sin(t))
        assert v == pytest.approx(b0 * r, rel=1e-13)


@pytest.mark.parametrize("a,s", [(0.5, 30.0), (3.0, 800.0)])
def test_potential_circular_dpie_closed_form(oracle, a, s):
    """psi(r) = F b0 [g(a) - g(s)], g(w) = sqrt(w^2+r^2) - w - w ln(w + sqrt(w^2+r^2)):
    the radial integral of the enclosed-mass deflection."""
    b0 = 11.0
    F = s / (s - a)
    for r in [1e-3, 0.4, 2.0, 17.0, 150.0, 3000.0]:
        t = RNG.uniform(0, 2 * math.pi)
        v, m = oracle.potential_eval(pot(0, 0, b0, 0.0, RNG.uniform(0, 3), a, s),
                                     r * math.cos(t), r * math.sin(t))
        with mp.workdps(50):
            R = mp.mpf(r)
            g = lambda w: mp.sqrt(w * w + R * R) - w - w * mp.log(w + mp.sqrt(w * w + R * R))
            ref = float(b0 * F * (g(mp.mpf(a)) - g(mp.mpf(s))))
        assert v == pytest.approx(ref, rel=1e-12, abs=1e-14 * m)


def test_potential_gradient_is_deflection(oracle):
    """Central differences of psi reproduce alpha (elliptical dPIEs)."""
    for _ in range(40):
        p = rand_pot()
        x, y = RNG.uniform(-40, 40, 2)
        h = 1e-5
        px = (oracle.potential_eval(p, x + h, y)[0] - oracle.potential_eval(p, x - h, y)[0]) / (2 * h)
        py = (oracle.potential_eval(p, x, y + h)[0] - oracle.potential_eval(p, x, y - h)[0]) / (2 * h)
        v, m = oracle.pot_eval(p, x, y)
        _, mp_ = oracle.potential_eval(p, x, y)
        tol = 1e-9 * max(m[0], m[1]) + 1e-10 * mp_ / h
        assert abs(px - v[0]) < tol and abs(py - v[1]) < tol


def test_potential_laplacian_is_twice_convergence(oracle):
    """Second differences of psi: Laplacian = Hxx + Hyy = 2 kappa."""
    for _ in range(30):
        p = rand_pot()
        x, y = RNG.uniform(-30, 30, 2)
        h = 2e-3
        c = oracle.potential_eval(p, x, y)[0]
        lap = (oracle.potential_eval(p, x + h, y)[0] + oracle.potential_eval(p, x - h, y)[0]
               + oracle.potential_eval(p, x, y + h)[0] + oracle.potential_eval(p, x, y - h)[0]
               - 4 * c) / (h * h)
        v, m = oracle.pot_eval(p, x, y)
        scale = m[2] + m[4] + 1e-13 * abs(c) / (h * h) * 1e3
        assert abs(lap - (v[2] + v[4])) < 1e-4 * scale


def test_time_delay_sis_images(oracle):
    """SIS scaled by f: the two images differ in arrival time by
    scale * 2 f b0 |beta|, and the time-delay surface is stationary at both."""
    b0, f, scale = 8.0, 0.7, 3.5
    lens = dict(x0=[0.0], y0=[0.0], b0=[b0], eps=[0.0], phi=[0.0], rcore=[0.0], rcut=[math.inf])
    for _ in range(10):
        r = RNG.uniform(0.1, 0.9) * f * b0
        t = RNG.uniform(0, 2 * math.pi)
        beta = (r * math.cos(t), r * math.sin(t))
        times = []
        for rad in (r + f * b0, r - f * b0):
            x, y = rad * math.cos(t), rad * math.sin(t)
            h = 1e-4
            pts = [(x, y), (x + h, y), (x - h, y), (x, y + h), (x, y - h)]
            xs = np.array([q[0] for q in pts])
            vals = []
            for q in pts:
                g = (1, 1, q[0], q[1], 1.0, 1.0)
                out, _ = oracle.potential_map(lens, g, f, beta, scale)
                vals.append(out[0, 0])
            times.append(vals[0])
            gx, gy = (vals[1] - vals[2]) / (2 * h), (vals[3] - vals[4]) / (2 * h)
            assert abs(gx) < 1e-6 * scale * b0 and abs(gy) < 1e-6 * scale * b0
        assert times[1] - times[0] == pytest.approx(scale * 2 * f * b0 * r, rel=1e-10)


def test_time_delay_scale_einstein_de_sitter(oracle):
    """Omega_m = 1: chi(z) = 2 (1 - 1/sqrt(1+z)) c/H0, so the scale is
    chi_l chi_s / ((chi_s - chi_l) H0) per rad^2."""
    h0 = 70.0
    for zl, zs in [(0.2, 1.0), (0.4, 2.0), (0.5, 5.0)]:
        cl, cs = (2 * (1 - 1 / math.sqrt(1 + z)) for z in (zl, zs))
        h0_si = h0 * 1000.0 / 3.0856775814913673e22
        want = cl * cs / ((cs - cl) * h0_si) * (math.pi / 648000.0) ** 2 / 86400.0
        assert oracle.time_delay_scale(zl, zs, h0, 1.0, 0.0) == pytest.approx(want, rel=1e-10)


# --------------------------------------------------------------------------
# Metropolis sampler
# --------------------------------------------------------------------------
def _sis_sampler_problem():
    """One SIS at the origin whose velocity dispersion is the only free
    parameter (the other six have zero step and a point prior), one system of
    three images: chi^2 is a smooth function of sigma with one minimum."""
    cat = dict(off=np.array([0, 3], np.int32), x=np.array([10.0, -6.0, 2.0]),
               y=np.array([1.0, 7.0, -9.0]), sig=np.array([0.5, 0.5, 0.5]), f=np.array([0.7]))
    base = np.array([0.0, 0.0, 700.0, 0.0, 0.0, 0.0, math.inf])
    return cat, base


def test_mcmc_zero_step_and_prior_rules(oracle):
    cat, base = _sis_sampler_problem()
    W = 6
    params = np.tile(base, (W, 1, 1)).astype(np.float64)
    params[:, 0, 2] = np.linspace(650.0, 750.0, W)
    chi2 = oracle.chi2_of_physical(empty_pots(), cat, params)
    acc = np.zeros(W, np.int32)
    lo = base.reshape(1, 7).copy()
    hi = base.reshape(1, 7).copy()
    lo[0, 2], hi[0, 2] = 600.0, 800.0
    step = np.zeros((1, 7))
    u = np.full((W, 8), 0.5)
    # zero step: the proposal is the current state, always accepted, nothing moves
    p0 = params.copy()
    assert oracle.mcmc_step(empty_pots(), cat, params, chi2, acc, lo, hi, step, u) == W
    assert np.array_equal(params, p0) and np.all(acc == 1)
    # a proposal beyond the prior box is rejected even when it lowers chi^2:
    # a box below the chi^2 minimum, walkers at its upper edge, moves upward
    g = np.tile(base, (301, 1, 1))
    g[:, 0, 2] = np.linspace(300.0, 1500.0, 301)
    smin = g[int(np.argmin(oracle.chi2_of_physical(empty_pots(), cat, g))), 0, 2]
    lo[0, 2], hi[0, 2] = smin - 300.0, smin - 100.0
    params[:, 0, 2] = smin - 110.0
    chi2 = oracle.chi2_of_physical(empty_pots(), cat, params)
    p0 = params.copy()
    step[0, 2] = 60.0
    u[:, 2] = 1.0  # sigma + 60: outside the box, closer to the minimum
    moved = params.copy()
    moved[:, 0, 2] += 60.0
    assert np.all(oracle.chi2_of_physical(empty_pots(), cat, moved) < chi2)
    assert oracle.mcmc_step(empty_pots(), cat, params, chi2, acc, lo, hi, step, u) == 0
    assert np.array_equal(params, p0)


def test_mcmc_acceptance_threshold(oracle):
    """A move that raises chi^2 by d is accepted exactly when -2 ln u > d."""
    cat, base = _sis_sampler_problem()
    lo, hi = base.reshape(1, 7).copy(), base.reshape(1, 7).copy()
    lo[0, 2], hi[0, 2] = 100.0, 2000.0
    sig_grid = np.linspace(300.0, 1500.0, 601)
    g = np.tile(base, (len(sig_grid), 1, 1))
    g[:, 0, 2] = sig_grid
    c = oracle.chi2_of_physical(empty_pots(), cat, g)
    i0 = int(np.argmin(c))
    start = sig_grid[i0]
    target = start + 40.0  # uphill move
    params = np.tile(base, (2, 1, 1))
    params[:, 0, 2] = start
    chi2 = oracle.chi2_of_physical(empty_pots(), cat, params)
    moved = params.copy()
    moved[:, 0, 2] = target
    d = float(oracle.chi2_of_physical(empty_pots(), cat, moved)[0] - chi2[0])
    assert d > 0.1
    step = np.zeros((1, 7))
    step[0, 2] = 40.0
    u = np.full((2, 8), 0.5)
    u[:, 2] = 1.0  # proposal = start + 40 exactly
    u[0, 7] = math.exp(-d / 2) * (1 - 1e-9)  # -2 ln u just above d: accept
    u[1, 7] = math.exp(-d / 2) * (1 + 1e-9)  # just below: reject
    acc = np.zeros(2, np.int32)
    oracle.mcmc_step(empty_pots(), cat, params, chi2, acc, lo, hi, step, u)
    assert list(acc) == [1, 0]
    assert params[0, 0, 2] == target and params[1, 0, 2] == start


def test_mcmc_samples_the_posterior(oracle):
    """Stationary distribution: after burn-in the walkers' sigma follows
    exp(-chi^2/2) on the prior box (chi^2 from the oracle on a fine grid,
    integrated by the trapezoid rule): mean within 5 standard errors of the
    4096 walkers, standard deviation within 12%."""
    cat, base = _sis_sampler_problem()
    sig_grid = np.linspace(300.0, 1500.0, 2401)
    g = np.tile(base, (len(sig_grid), 1, 1))
    g[:, 0, 2] = sig_grid
    c = oracle.chi2_of_physical(empty_pots(), cat, g)
    imin = int(np.argmin(c))
    wgt = np.exp(-(c - c[imin]) / 2)
    # prior box: +-6 posterior widths around the minimum
    mean0 = np.trapezoid(wgt * sig_grid, sig_grid) / np.trapezoid(wgt, sig_grid)
    sd0 = math.sqrt(np.trapezoid(wgt * (sig_grid - mean0) ** 2, sig_grid) / np.trapezoid(wgt, sig_grid))
    lo_s, hi_s = mean0 - 6 * sd0, mean0 + 6 * sd0
    inside = (sig_grid >= lo_s) & (sig_grid <= hi_s)
    sg, wg = sig_grid[inside], wgt[inside]
    mean = np.trapezoid(wg * sg, sg) / np.trapezoid(wg, sg)
    sd = math.sqrt(np.trapezoid(wg * (sg - mean) ** 2, sg) / np.trapezoid(wg, sg))
    W, steps = 4096, 250
    rng = np.random.default_rng(11)
    params = np.tile(base, (W, 1, 1))
    params[:, 0, 2] = rng.uniform(lo_s, hi_s, W)
    chi2 = oracle.chi2_of_physical(empty_pots(), cat, params)
    acc = np.zeros(W, np.int32)
    lo, hi = base.reshape(1, 7).copy(), base.reshape(1, 7).copy()
    lo[0, 2], hi[0, 2] = lo_s, hi_s
    step = np.zeros((1, 7))
    step[0, 2] = 2.5 * sd
    for _ in range(steps):
        u = 1.0 - rng.random((W, 8))  # (0, 1]
        oracle.mcmc_step(empty_pots(), cat, params, chi2, acc, lo, hi, step, u)
    s = params[:, 0, 2]
    assert abs(s.mean() - mean) < 5 * sd / math.sqrt(W)
    assert abs(s.std() / sd - 1) < 0.12
    assert 0.1 < acc.mean() / steps < 0.9
