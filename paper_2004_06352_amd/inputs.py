"""Seeded synthetic inputs for the lens-gradient hot path.

This module only draws random numbers and lays them out.  It holds none of the
lensing arithmetic: potentials are described by their *physical* parameters
(centre, velocity dispersion, Lenstool ellipticity, angle, core and cut radii)
and constraint systems by their positions, errors and source redshifts.  Each
consumer converts these to the deflection-amplitude form on its own.

The paper's lens models (MACS J1149 with 217 potentials and 80 sources / 227
images on a 5000^2 grid over 150 arcsec, Sec. 5; Abell 2744 with 258
potentials on 6000^2 maps, Sec. 2.4) are not available; these generators stand
in for them with the same kinds of shapes: one or two cluster-scale halos plus
hundreds of galaxy-scale halos, multiple-image systems of 2-5 images, grids of
10^5-10^7 points.

Conventions
  pots   dict of float64 arrays, one entry per dPIE:
           x0, y0  centre [arcsec]; sigma  velocity dispersion [km/s];
           e       ellipticity (a^2-b^2)/(a^2+b^2); phi  position angle [rad];
           rcore, rcut  [arcsec] (rcut may be inf)
  grid   (nx, ny, x0, y0, dx, dy): point (i, j) = (x0 + i dx, y0 + j dy)
  catalog dict: off int32 [nsys+1]; x, y, sig float64 [nimg]; zs float64 [nsys]
"""
from __future__ import annotations

import math
import os

import numpy as np

PHYS_KEYS = ("x0", "y0", "sigma", "e", "phi", "rcore", "rcut")
ZL = 0.4

_HERE = os.path.dirname(os.path.abspath(__file__))
CATALOG_PATH = os.path.join(_HERE, "data", "cfg3_catalog.txt")


def pixel_centre_grid(n: int, lo: float, hi: float):
    """n x n pixel centres covering [lo, hi]^2."""
    d = (hi - lo) / n
    return (n, n, lo + 0.5 * d, lo + 0.5 * d, d, d)


def _table(rows):
    """list of (x0, y0, sigma, e, phi, rcore, rcut) -> dict of arrays."""
    arr = np.asarray(rows, dtype=np.float64).reshape(-1, 7)
    return {k: np.ascontiguousarray(arr[:, i]) for i, k in enumerate(PHYS_KEYS)}


def concat(*tables):
    return {k: np.concatenate([t[k] for t in tables]) for k in PHYS_KEYS}


def take(t, idx):
    return {k: np.ascontiguousarray(t[k][idx]) for k in PHYS_KEYS}


def schechter_luminosities(rng, n, alpha=-1.1, lo=0.01, hi=10.0):
    """L/L* drawn from p(L) ~ L^alpha exp(-L) on [lo, hi]: power-law proposal
    by inverse CDF, accepted with probability exp(-L)."""
    out = np.empty(0)
    a1 = alpha + 1.0
    while out.size < n:
        u = rng.random(2 * n)
        L = (lo ** a1 + u * (hi ** a1 - lo ** a1)) ** (1.0 / a1)
        keep = rng.random(L.size) < np.exp(-L)
        out = np.concatenate([out, L[keep]])
    return out[:n]


def galaxies(rng, n, lo, hi, sigma_star=180.0, rcut_star=8.0, rcore_star=0.05):
    """Galaxy-scale dPIEs with sigma ~ L^(1/4), rcut and rcore ~ L^(1/2)."""
    L = schechter_luminosities(rng, n)
    x0 = rng.uniform(lo, hi, n)
    y0 = rng.uniform(lo, hi, n)
    e = rng.uniform(0.0, 0.5, n)
    phi = rng.uniform(0.0, math.pi, n)
    sig = sigma_star * L ** 0.25
    rcut = rcut_star * L ** 0.5
    rcore = rcore_star * L ** 0.5
    return _table(np.stack([x0, y0, sig, e, phi, rcore, rcut], axis=1))


CLUSTER1 = (0.0, 0.0, 1000.0, 0.3, math.pi / 6, 5.0, 1000.0)
CLUSTER2 = (40.0, -25.0, 700.0, 0.2, -math.pi / 5, 3.0, 800.0)


def config1(seed=1):
    """256^2 pixel centres over [-100, 100]^2; one cluster dPIE plus 20 galaxy
    dPIEs (sigma 50-250 km/s, e 0-0.5, rcore 0.05, rcut 10-50); zl 0.4, zs 2."""
    rng = np.random.default_rng(seed)
    n = 20
    rows = [CLUSTER1]
    sig = rng.uniform(50, 250, n)
    e = rng.uniform(0, 0.5, n)
    phi = rng.uniform(0, math.pi, n)
    rcut = rng.uniform(10, 50, n)
    x0 = rng.uniform(-100, 100, n)
    y0 = rng.uniform(-100, 100, n)
    for k in range(n):
        rows.append((x0[k], y0[k], sig[k], e[k], phi[k], 0.05, rcut[k]))
    return dict(name="cfg1_256sq_21pot", pots=_table(rows),
                grid=pixel_centre_grid(256, -100.0, 100.0), zl=ZL, zs=2.0)


def config2(seed=2, n=2048, n_gal=500):
    """2048^2 over [-100, 100]^2; two cluster dPIEs + 500 Schechter galaxies."""
    rng = np.random.default_rng(seed)
    pots = concat(_table([CLUSTER1, CLUSTER2]), galaxies(rng, n_gal, -100.0, 100.0))
    return dict(name=f"cfg2_{n}sq_{2 + n_gal}pot", pots=pots,
                grid=pixel_centre_grid(n, -100.0, 100.0), zl=ZL, zs=2.0)


def config_p(seed=7, n=5000, n_gal=215):
    """The shape of the paper's headline map (Sec. 5: a 5000^2 grid over
    150 arcsec, 217 potentials): 5000^2 pixel centres over [-75, 75]^2, the
    two cluster dPIEs of workload 2 plus 215 Schechter galaxies over the
    field.  The paper's lens model itself is not available; this stands in
    for its sizes only."""
    rng = np.random.default_rng(seed)
    pots = concat(_table([CLUSTER1, CLUSTER2]), galaxies(rng, n_gal, -75.0, 75.0))
    return dict(name=f"cfgP_{n}sq_{2 + n_gal}pot", pots=pots,
                grid=pixel_centre_grid(n, -75.0, 75.0), zl=ZL, zs=2.0)


# --- the config-3 model: 6 free dPIEs with uniform priors + 300 fixed galaxies
# (lo, hi) per physical parameter in PHYS_KEYS order
_FREE_PRIORS = [
    # halo A
    ((-3, 3), (-3, 3), (800, 1200), (0.1, 0.5), (0, math.pi), (3, 10), (800, 1500)),
    # halo B
    ((30, 40), (-25, -15), (400, 800), (0.0, 0.5), (0, math.pi), (1, 6), (300, 1000)),
    # BCG
    ((-1, 1), (-1, 1), (200, 400), (0.0, 0.4), (0, math.pi), (0.01, 0.3), (20, 100)),
]
_FREE_GAL_CENTRES = [(14.0, 9.0), (-17.0, 21.0), (23.0, -31.0)]
for _cx, _cy in _FREE_GAL_CENTRES:
    _FREE_PRIORS.append(((_cx - 1, _cx + 1), (_cy - 1, _cy + 1), (100, 300), (0.0, 0.5),
                         (0, math.pi), (0.01, 0.2), (5, 50)))
N_FREE = len(_FREE_PRIORS)


def free_priors():
    return [tuple(p) for p in _FREE_PRIORS]


def truth_free():
    """The config-3 'true' free potentials: prior midpoints."""
    return _table([[0.5 * (lo + hi) for lo, hi in pr] for pr in _FREE_PRIORS])


def fixed_galaxies(seed=3, n=300):
    rng = np.random.default_rng(1000 + seed)
    return galaxies(rng, n, -75.0, 75.0)


def draw_samples(rng, n_samples, uneven=False):
    """n_samples draws of the free potentials from their uniform priors.
    Returns (free table concatenated over samples, free_off int32 [S+1]).
    uneven=True keeps the three halos and a random subset (0-3, order kept) of
    the three free galaxies in each sample, so sample sizes differ (3-6)."""
    lo = np.array([[p[0] for p in pr] for pr in _FREE_PRIORS])
    hi = np.array([[p[1] for p in pr] for pr in _FREE_PRIORS])
    draw = lo + rng.random((n_samples, N_FREE, 7)) * (hi - lo)
    if uneven:
        keep = np.ones((n_samples, N_FREE), dtype=bool)
        keep[:, 3:] = rng.random((n_samples, N_FREE - 3)) < 0.5
    else:
        keep = np.ones((n_samples, N_FREE), dtype=bool)
    rows = draw[keep]
    off = np.concatenate([[0], np.cumsum(keep.sum(axis=1))]).astype(np.int32)
    return _table(rows), off


def load_catalog(path=CATALOG_PATH):
    """The config-3 constraint catalogue (stored text file; see its header)."""
    if not os.path.exists(path):
        raise FileNotFoundError(f"constraint catalogue missing: {path}")
    sys_id, zs, x, y, sig, x_true, y_true = [], [], [], [], [], [], []
    with open(path) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            t = line.split()
            sys_id.append(int(t[0]))
            zs.append(float(t[1]))
            x.append(float(t[2]))
            y.append(float(t[3]))
            sig.append(float(t[4]))
            x_true.append(float(t[5]))
            y_true.append(float(t[6]))
    sys_id = np.asarray(sys_id)
    nsys = int(sys_id.max()) + 1
    counts = np.bincount(sys_id, minlength=nsys)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    zsys = np.zeros(nsys)
    zsys[sys_id] = zs
    return dict(off=off, x=np.asarray(x), y=np.asarray(y), sig=np.asarray(sig), zs=zsys,
                x_true=np.asarray(x_true), y_true=np.asarray(y_true))


def config3(seed=3, n_samples=4096, uneven=False):
    """4096 MCMC samples of 6 free dPIEs (uniform priors) + 300 fixed galaxies;
    60 multiple-image systems with 2-5 images each."""
    rng = np.random.default_rng(seed)
    free, off = draw_samples(rng, n_samples, uneven=uneven)
    return dict(name=f"cfg3_{n_samples}samples", fixed=fixed_galaxies(seed), free=free,
                free_off=off, catalog=load_catalog(), zl=ZL)


def sampler_start(seed=3, n_walkers=4096, step_frac=0.02):
    """Walkers for the Metropolis sampler on the config-3 model: starting
    points drawn from the uniform priors of the 6 free dPIEs, the prior box,
    and proposal half-widths step_frac of each prior's width.  Returns a dict:
    params (W, 6, 7), lo, hi, step (6, 7), fixed, catalog, zl."""
    rng = np.random.default_rng(7000 + seed)
    lo = np.array([[p[0] for p in pr] for pr in _FREE_PRIORS], dtype=np.float64)
    hi = np.array([[p[1] for p in pr] for pr in _FREE_PRIORS], dtype=np.float64)
    params = lo + rng.random((n_walkers, N_FREE, 7)) * (hi - lo)
    return dict(name=f"cfg3_{n_walkers}walkers", params=np.ascontiguousarray(params), lo=lo,
                hi=hi, step=step_frac * (hi - lo), fixed=fixed_galaxies(seed),
                catalog=load_catalog(), zl=ZL)


def sampler_uniforms(rng, n_walkers, n_free):
    """One step's uniforms in (0, 1]: 7 n_free for the proposal, 1 for the
    acceptance test, per walker."""
    return np.ascontiguousarray(1.0 - rng.random((n_walkers, 7 * n_free + 1)))


def config4(seed=3, n_samples=512, n=1000):
    """1000^2 pixel-centre vertices over [-75, 75]^2; the first 512 samples of
    the config-3 model and catalogue."""
    c3 = config3(seed=seed, n_samples=n_samples)
    c3["name"] = f"cfg4_{n}sq_{n_samples}samples"
    c3["grid"] = pixel_centre_grid(n, -75.0, 75.0)
    return c3


def config5_models(seed=5, n_models=32, pot_range=(50, 1000)):
    """Pool of lens models served by map requests: potential counts
    log-uniform in pot_range (config-2 generator).  Returns [(npot, seed)]."""
    rng = np.random.default_rng(seed + 1000)
    out = []
    for _ in range(n_models):
        npot = int(round(math.exp(rng.uniform(math.log(pot_range[0]), math.log(pot_range[1])))))
        out.append((npot, int(rng.integers(1 << 30))))
    return out


def config5_requests(seed=5, n_requests=2000, rate_hz=10.0,
                     map_sides=(512, 1024, 2048, 4096), n_models=32, pot_range=(50, 1000),
                     batch_range=(64, 4096)):
    """Poisson stream of mixed requests: half lensing maps (side from
    map_sides, model drawn from a pool of n_models lens models with potential
    counts log-uniform in pot_range), half chi^2 batches (size log-uniform in
    batch_range, config-3 model, fresh samples per request).  Returns a list of
    dicts with arrival time t [s]."""
    rng = np.random.default_rng(seed)
    models = config5_models(seed, n_models, pot_range)
    t, reqs = 0.0, []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        if rng.random() < 0.5:
            side = int(rng.choice(map_sides))
            mid = int(rng.integers(n_models))
            reqs.append(dict(id=r, t=t, kind="map", side=side, model=mid,
                             npot=models[mid][0], model_seed=models[mid][1]))
        else:
            bs = int(round(math.exp(rng.uniform(math.log(batch_range[0]),
                                                math.log(batch_range[1])))))
            reqs.append(dict(id=r, t=t, kind="chi2", samples=bs,
                             seed=int(rng.integers(1 << 30))))
    return reqs


def map_request_pots(npot, seed):
    """Potentials of one map request: the two cluster halos + Schechter galaxies."""
    rng = np.random.default_rng(seed)
    base = _table([CLUSTER1, CLUSTER2])
    if npot <= 2:
        return take(base, np.arange(npot))
    return concat(base, galaxies(rng, npot - 2, -100.0, 100.0))
