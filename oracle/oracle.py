"""Python access to the FP64 CPU oracle (``lens_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference the GPU
library is checked against; only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It shares nothing with the GPU
library beyond the seeded input dictionaries both are fed.

Inputs use plain numpy containers:
  pots     dict of equal-length float64 arrays x0, y0, b0, eps, phi, rcore, rcut
           (a dPIE per entry; b0 is the amplitude at Dls/Ds = 1, rcut may be inf)
  grid     (nx, ny, x0, y0, dx, dy); point (i, j) = (x0 + i dx, y0 + j dy)
  catalog  dict: off int32 [nsys+1], x, y, sig float64 [nimg], f float64 [nsys]
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lens_oracle.c")
LIB = os.path.join(HERE, "liblens_oracle.so")

CFLAGS = ["-O2", "-std=gnu11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wno-unused-variable"]

POT_KEYS = ("x0", "y0", "b0", "eps", "phi", "rcore", "rcut")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FMA contraction off)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


class _Pots(C.Structure):
    _fields_ = [("n", C.c_int)] + [(k, C.POINTER(C.c_double)) for k in POT_KEYS]


class _Cat(C.Structure):
    _fields_ = [("nsys", C.c_int), ("off", C.POINTER(C.c_int)),
                ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("sig", C.POINTER(C.c_double)), ("f", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.or_pot_eval.argtypes = [dp, C.c_double, C.c_double, dp, dp]
        L.or_eval_points.argtypes = [C.POINTER(_Pots), C.c_int, dp, dp, dp, dp]
        L.or_map.argtypes = [C.POINTER(_Pots), C.c_int, C.c_int, C.c_double, C.c_double,
                             C.c_double, C.c_double, C.c_double, dp, dp]
        L.or_dlsds.argtypes = [C.c_double] * 4 + [dp]
        L.or_dlsds.restype = C.c_int
        L.or_unlens.argtypes = [C.POINTER(_Pots), C.POINTER(_Pots), ip, C.c_int,
                                C.POINTER(_Cat), dp, dp, dp]
        L.or_chi2_source.argtypes = [C.POINTER(_Pots), C.POINTER(_Pots), ip, C.c_int,
                                     C.POINTER(_Cat), dp]
        L.or_sources.argtypes = [C.POINTER(_Pots), C.POINTER(_Pots), ip, C.c_int,
                                 C.POINTER(_Cat), dp, dp]
        L.or_orient_exact.argtypes = [C.c_double] * 6
        L.or_orient_exact.restype = C.c_int
        L.or_orient_perturbed.argtypes = [C.c_double] * 6
        L.or_orient_perturbed.restype = C.c_int
        L.or_find_images.argtypes = [dp, dp, C.c_int, C.c_int] + [C.c_double] * 7 + [
            C.c_int, C.POINTER(C.c_longlong), dp, dp]
        L.or_find_images.restype = C.c_int
        L.or_assign_system.argtypes = [C.c_int, dp, dp, C.c_int, dp, dp, dp, C.c_double, ip]
        L.or_assign_system.restype = C.c_double
        L.or_chi2_image.argtypes = [C.POINTER(_Pots), C.POINTER(_Pots), ip, C.c_int, C.c_int,
                                    C.POINTER(_Cat), dp, dp, C.c_int, C.c_int,
                                    C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_int, C.c_double, dp, ip, ip, dp, dp,
                                    C.POINTER(C.c_longlong), C.c_int, C.c_double, C.c_double,
                                    ip]
        L.or_refine_image.argtypes = [C.POINTER(_Pots), C.POINTER(_Pots), C.c_int, C.c_int,
                                      C.c_double, C.c_double, C.c_double, dp, dp, C.c_int,
                                      C.c_double, C.c_double]
        L.or_refine_image.restype = C.c_int
        L.or_chi2_image.restype = C.c_int
        L.or_edge_margin.argtypes = [dp, dp, C.c_int, C.c_int] + [C.c_double] * 7
        L.or_edge_margin.restype = C.c_double
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None else None


class _Keep:
    """Holds the numpy arrays a ctypes struct points into."""

    def __init__(self):
        self.refs = []

    def d(self, a):
        a = _d(a)
        self.refs.append(a)
        return a


def _pots(p, keep):
    arrs = [keep.d(p[k]) for k in POT_KEYS]
    n = len(arrs[0])
    assert all(len(a) == n for a in arrs)
    return _Pots(n, *[_ptr(a) for a in arrs])


def _cat(cat, keep):
    off = np.ascontiguousarray(cat["off"], dtype=np.int32)
    keep.refs.append(off)
    return _Cat(len(off) - 1, _ptr(off, C.c_int), _ptr(keep.d(cat["x"])),
                _ptr(keep.d(cat["y"])), _ptr(keep.d(cat["sig"])), _ptr(keep.d(cat["f"])))


def pot_eval(p7, x, y):
    """One potential (x0, y0, b0, eps, phi, rcore, rcut) at (x, y) -> (val[5], mag[5])."""
    p = _d(p7)
    v, m = np.zeros(5), np.zeros(5)
    lib().or_pot_eval(_ptr(p), float(x), float(y), _ptr(v), _ptr(m))
    return v, m


def eval_points(pots, x, y):
    """Sum over potentials at points, Dls/Ds = 1 -> (val[5, n], mag[5, n])."""
    keep = _Keep()
    P = _pots(pots, keep)
    x, y = keep.d(np.ravel(x)), keep.d(np.ravel(y))
    out, mag = np.zeros((5, len(x))), np.zeros((5, len(x)))
    lib().or_eval_points(C.byref(P), len(x), _ptr(x), _ptr(y), _ptr(out), _ptr(mag))
    return out, mag


def lens_map(pots, grid, dlsds=1.0, want_mag=True):
    """Five-channel map [ax, ay, hxx, hxy, hyy] of shape (5, ny, nx), plus its scale."""
    nx, ny, gx0, gy0, dx, dy = grid
    keep = _Keep()
    P = _pots(pots, keep)
    out = np.zeros((5, ny, nx))
    mag = np.zeros((5, ny, nx)) if want_mag else None
    lib().or_map(C.byref(P), nx, ny, gx0, gy0, dx, dy, float(dlsds), _ptr(out),
                 _ptr(mag) if mag is not None else None)
    return out, mag


def potential_eval(p7, x, y):
    """Lensing potential of one potential {x0, y0, b0, eps, phi, rcore, rcut}
    at (x, y), Dls/Ds = 1 -> (value, magnitude scale)."""
    L = lib()
    L.or_potential.argtypes = [C.POINTER(C.c_double), C.c_double, C.c_double,
                               C.POINTER(C.c_double)]
    L.or_potential.restype = C.c_double
    p = _d(np.asarray(p7, dtype=np.float64))
    m = C.c_double()
    v = L.or_potential(_ptr(p), float(x), float(y), C.byref(m))
    return v, m.value


def potential_map(pots, grid, dlsds=1.0, beta=(0.0, 0.0), scale=0.0):
    """Potential map (scale == 0) or time-delay surface scale (|theta-beta|^2/2
    - psi) of shape (ny, nx), plus its magnitude scale."""
    nx, ny, gx0, gy0, dx, dy = grid
    keep = _Keep()
    P = _pots(pots, keep)
    out = np.zeros((ny, nx))
    mag = np.zeros((ny, nx))
    L = lib()
    L.or_potential_map.argtypes = [C.POINTER(_Pots), C.c_int, C.c_int] + [C.c_double] * 8 + \
        [C.POINTER(C.c_double)] * 2
    L.or_potential_map.restype = None
    L.or_potential_map(C.byref(P), nx, ny, gx0, gy0, dx, dy, float(dlsds), float(beta[0]),
                       float(beta[1]), float(scale), _ptr(out), _ptr(mag))
    return out, mag


def time_delay_scale(zl, zs, h0=70.0, om=0.3, ol=0.7):
    """(1 + zl) Dl Ds / (c Dls) in days per arcsec^2 (flat cosmology)."""
    L = lib()
    L.or_time_delay_scale.argtypes = [C.c_double] * 5
    L.or_time_delay_scale.restype = C.c_double
    return L.or_time_delay_scale(float(zl), float(zs), float(h0), float(om), float(ol))


def mcmc_step(fixed, cat, params, chi2, accepted, lo, hi, step, u, convention=0):
    """One Metropolis step of every walker, in place (see lens_oracle.c).
    params (W, nfree, 7) physical, chi2 (W,), accepted (W,) int32, lo/hi/step
    (nfree, 7), u (W, 7 nfree + 1) in (0, 1].  Returns the accepted count."""
    for a_ in (params, chi2, lo, hi, step, u):
        assert a_.dtype == np.float64 and a_.flags.c_contiguous
    assert accepted.dtype == np.int32 and accepted.flags.c_contiguous
    W, nfree = params.shape[0], params.shape[1]
    keep = _Keep()
    Pf, Cc = _pots(fixed, keep), _cat(cat, keep)
    L = lib()
    L.or_mcmc_step.argtypes = [C.POINTER(_Pots), C.POINTER(_Cat), C.c_int, C.c_int,
                               C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.POINTER(C.c_int)] + [C.POINTER(C.c_double)] * 4 + [C.c_int]
    L.or_mcmc_step.restype = C.c_int
    return L.or_mcmc_step(C.byref(Pf), C.byref(Cc), W, nfree, _ptr(params), _ptr(chi2),
                          _ptr(accepted, C.c_int), _ptr(lo), _ptr(hi), _ptr(step), _ptr(u),
                          int(convention))


def chi2_of_physical(fixed, cat, params, convention=0):
    """Source-plane chi^2 of walkers given as physical parameters (W, nfree, 7)."""
    W, nfree = params.shape[0], params.shape[1]
    flat = params.reshape(W * nfree, 7)
    phys = {k: np.ascontiguousarray(flat[:, i]) for i, k in
            enumerate(("x0", "y0", "sigma", "e", "phi", "rcore", "rcut"))}
    free = phys_to_pots(phys, convention)
    off = (np.arange(W + 1) * nfree).astype(np.int32)
    return chi2_source(fixed, free, off, cat)


def derived(hxx, hxy, hyy):
    """kappa, gamma1, gamma2, gamma, det (of the inverse magnification matrix)
    and mu from a summed second-derivative map (see lens_oracle.c)."""
    hxx, hxy, hyy = (np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (hxx, hxy, hyy))
    shape = hxx.shape
    n = hxx.size
    outs = {k: np.zeros(n) for k in ("kappa", "gamma1", "gamma2", "gamma", "det", "mu")}
    L = lib()
    L.or_derived.argtypes = [C.c_long] + [C.POINTER(C.c_double)] * 9
    L.or_derived.restype = None
    L.or_derived(n, _ptr(hxx), _ptr(hxy), _ptr(hyy), _ptr(outs["kappa"]), _ptr(outs["gamma1"]),
                 _ptr(outs["gamma2"]), _ptr(outs["gamma"]), _ptr(outs["det"]), _ptr(outs["mu"]))
    return {k: v.reshape(shape) for k, v in outs.items()}


def dlsds(zl, zs, om=0.3, ol=0.7):
    out = C.c_double()
    rc = lib().or_dlsds(float(zl), float(zs), float(om), float(ol), C.byref(out))
    if rc != 0:
        raise ValueError("invalid redshifts or non-flat cosmology")
    return out.value


def _model_args(fixed, free, free_off, keep):
    Pf, Pv = _pots(fixed, keep), _pots(free, keep)
    off = np.ascontiguousarray(free_off, dtype=np.int32)
    keep.refs.append(off)
    return Pf, Pv, off


def unlens(fixed, free, free_off, m, cat):
    """beta_ij of sample m -> (bx, by, sabs) per image."""
    keep = _Keep()
    Pf, Pv, off = _model_args(fixed, free, free_off, keep)
    Cc = _cat(cat, keep)
    n = int(cat["off"][-1])
    bx, by, sabs = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().or_unlens(C.byref(Pf), C.byref(Pv), _ptr(off, C.c_int), int(m), C.byref(Cc),
                    _ptr(bx), _ptr(by), _ptr(sabs))
    return bx, by, sabs


def sources(fixed, free, free_off, m, cat):
    keep = _Keep()
    Pf, Pv, off = _model_args(fixed, free, free_off, keep)
    Cc = _cat(cat, keep)
    ns = len(cat["off"]) - 1
    sx, sy = np.zeros(ns), np.zeros(ns)
    lib().or_sources(C.byref(Pf), C.byref(Pv), _ptr(off, C.c_int), int(m), C.byref(Cc),
                     _ptr(sx), _ptr(sy))
    return sx, sy


def chi2_source(fixed, free, free_off, cat):
    keep = _Keep()
    Pf, Pv, off = _model_args(fixed, free, free_off, keep)
    Cc = _cat(cat, keep)
    ns = len(off) - 1
    out = np.zeros(ns)
    lib().or_chi2_source(C.byref(Pf), C.byref(Pv), _ptr(off, C.c_int), ns, C.byref(Cc),
                         _ptr(out))
    return out


def orient_exact(ax, ay, bx, by, px, py):
    return lib().or_orient_exact(ax, ay, bx, by, px, py)


def orient_perturbed(ax, ay, bx, by, px, py):
    return lib().or_orient_perturbed(ax, ay, bx, by, px, py)


def find_images(ax, ay, grid, f, px, py, kmax=64):
    """Images of source (px, py) for one system -> (n, tri, x, y) (first kmax stored)."""
    nx, ny, gx0, gy0, dx, dy = grid
    ax, ay = _d(ax).reshape(-1), _d(ay).reshape(-1)
    assert ax.size == nx * ny and ay.size == nx * ny
    tri = np.zeros(max(kmax, 1), dtype=np.int64)
    ix, iy = np.zeros(max(kmax, 1)), np.zeros(max(kmax, 1))
    n = lib().or_find_images(_ptr(ax), _ptr(ay), nx, ny, gx0, gy0, dx, dy, float(f),
                             float(px), float(py), kmax,
                             tri.ctypes.data_as(C.POINTER(C.c_longlong)), _ptr(ix), _ptr(iy))
    k = min(n, kmax)
    return n, tri[:k], ix[:k], iy[:k]


def assign_system(ix, iy, cx, cy, sig, penalty):
    ix, iy, cx, cy, sig = map(_d, (ix, iy, cx, cy, sig))
    miss = C.c_int()
    part = lib().or_assign_system(len(ix), _ptr(ix), _ptr(iy), len(cx), _ptr(cx), _ptr(cy),
                                  _ptr(sig), float(penalty), C.byref(miss))
    return part, miss.value


def alpha_grid(pots, grid):
    """Deflection (Dls/Ds = 1) at every grid vertex -> (ax, ay) of shape (ny, nx)."""
    out, _ = lens_map(pots, grid, 1.0, want_mag=False)
    return out[0], out[1]


def chi2_image(fixed, free, free_off, cat, grid, m0=0, m1=None, kmax=16,
               penalty=0.0, alpha_fix=None, refine=None):
    """Image-plane chi^2 of samples [m0, m1) -> dict of arrays (see lens_oracle.c).
    refine = (max_iter, tol, max_shift) refines every stored image by Newton's
    method before the assignment; `nfail` counts images left at the grid
    estimate."""
    nx, ny, gx0, gy0, dx, dy = grid
    if m1 is None:
        m1 = len(free_off) - 1
    if alpha_fix is None:
        alpha_fix = alpha_grid(fixed, grid)
    keep = _Keep()
    Pf, Pv, off = _model_args(fixed, free, free_off, keep)
    Cc = _cat(cat, keep)
    afx, afy = keep.d(alpha_fix[0]).reshape(-1), keep.d(alpha_fix[1]).reshape(-1)
    S, ns = m1 - m0, len(cat["off"]) - 1
    chi2 = np.zeros(S)
    nimg = np.zeros((S, ns), dtype=np.int32)
    nmiss = np.zeros(S, dtype=np.int32)
    ix = np.zeros((S, ns, kmax))
    iy = np.zeros((S, ns, kmax))
    itri = np.full((S, ns, kmax), -1, dtype=np.int64)
    nfail = np.zeros(S, dtype=np.int32)
    it, tol, shift = refine if refine is not None else (0, 0.0, 0.0)
    over = lib().or_chi2_image(C.byref(Pf), C.byref(Pv), _ptr(off, C.c_int), m0, m1,
                               C.byref(Cc), _ptr(afx), _ptr(afy), nx, ny, gx0, gy0, dx, dy,
                               kmax, float(penalty), _ptr(chi2), _ptr(nimg, C.c_int),
                               _ptr(nmiss, C.c_int), _ptr(ix), _ptr(iy),
                               itri.ctypes.data_as(C.POINTER(C.c_longlong)), int(it),
                               float(tol), float(shift), _ptr(nfail, C.c_int))
    return dict(chi2=chi2, nimg=nimg, nmiss=nmiss, x=ix, y=iy, tri=itri, overflow=over,
                nfail=nfail)


def refine_image(fixed, free, f, beta, theta, max_iter=20, tol=1e-10, max_shift=1.0):
    """Newton refinement of one image position theta for the source beta with
    Dls/Ds f; the model is the fixed potentials plus `free` (all of it).
    Returns (x, y, iterations or -1)."""
    keep = _Keep()
    Pf, Pv = _pots(fixed, keep), _pots(free, keep)
    x, y = C.c_double(float(theta[0])), C.c_double(float(theta[1]))
    n = len(np.atleast_1d(free["x0"]))
    it = lib().or_refine_image(C.byref(Pf), C.byref(Pv), 0, n, float(f), float(beta[0]),
                               float(beta[1]), C.byref(x), C.byref(y), int(max_iter), float(tol),
                               float(max_shift))
    return x.value, y.value, it


def edge_margin(ax, ay, grid, f, px, py):
    nx, ny, gx0, gy0, dx, dy = grid
    ax, ay = _d(ax).reshape(-1), _d(ay).reshape(-1)
    return lib().or_edge_margin(_ptr(ax), _ptr(ay), nx, ny, gx0, gy0, dx, dy, float(f),
                                float(px), float(py))


def b0_from_sigma(sigma, convention=0):
    L = lib()
    L.or_b0_from_sigma.argtypes = [C.c_double, C.c_int]
    L.or_b0_from_sigma.restype = C.c_double
    return np.array([L.or_b0_from_sigma(float(s), int(convention)) for s in np.ravel(sigma)])


def eps_from_e(e):
    L = lib()
    L.or_eps_from_e.argtypes = [C.c_double]
    L.or_eps_from_e.restype = C.c_double
    return np.array([L.or_eps_from_e(float(v)) for v in np.ravel(e)])


def phys_to_pots(phys, convention=0):
    """Physical table (x0, y0, sigma, e, phi, rcore, rcut) -> oracle pots dict."""
    return dict(x0=_d(phys["x0"]), y0=_d(phys["y0"]),
                b0=b0_from_sigma(phys["sigma"], convention), eps=eps_from_e(phys["e"]),
                phi=_d(phys["phi"]), rcore=_d(phys["rcore"]), rcut=_d(phys["rcut"]))


def catalog_f(cat, zl, om=0.3, ol=0.7):
    """Catalogue dict with the per-system Dls/Ds filled in from its source redshifts."""
    out = dict(cat)
    out["f"] = np.array([dlsds(zl, z, om, ol) for z in cat["zs"]])
    return out
