"""Write ``paper_2004_06352_amd/data/cfg3_catalog.txt``: the multiple-image
constraint catalogue of the config-3 lens model (6 free dPIEs at their prior
midpoints + 300 fixed galaxy dPIEs, zl = 0.4).

Uses the oracle only (test infrastructure):
  1. deflection of the true model on a 1500^2 pixel-centre grid over [-75, 75]^2;
  2. sources drawn uniformly in [-15, 15]^2 with zs ~ U[1, 6];
  3. images by brute-force grid inversion (paper Sec. 2.3), each refined by
     Newton's method on the lens equation beta = theta - f alpha(theta)
     (Sec. 2.1, Eq. (1)) with the analytic Hessian, to |residual| < 1e-10";
  4. a system is kept when it has 2-5 distinct images, all inside
     [-70, 70]^2 and none within |det A^-1| < 0.05 of a critical line;
  5. 0.05" Gaussian noise is added to every image position (sigma = 0.05").

Run from the repository root:  python tests/golden/make_cfg3_catalog.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2004_06352_amd import inputs  # noqa: E402

OUT = os.path.join(ROOT, "paper_2004_06352_amd", "data", "cfg3_catalog.txt")
N_SYS = 60
SIGMA = 0.05


def newton(pots, f, beta, th):
    th = np.array(th, dtype=np.float64)
    for _ in range(60):
        v, _ = O.eval_points(pots, th[:, 0], th[:, 1])
        g = th - f * v[:2].T - beta
        if np.max(np.abs(g)) < 1e-11:
            break
        J11, J12, J22 = 1 - f * v[2], -f * v[3], 1 - f * v[4]
        det = J11 * J22 - J12 * J12
        th = th - np.stack([(J22 * g[:, 0] - J12 * g[:, 1]) / det,
                            (-J12 * g[:, 0] + J11 * g[:, 1]) / det], axis=1)
    v, _ = O.eval_points(pots, th[:, 0], th[:, 1])
    g = th - f * v[:2].T - beta
    det = (1 - f * v[2]) * (1 - f * v[4]) - (f * v[3]) ** 2
    return th, np.max(np.abs(g), axis=1), det


def main():
    truth = inputs.concat(inputs.fixed_galaxies(3), inputs.truth_free())
    pots = O.phys_to_pots(truth)
    grid = inputs.pixel_centre_grid(1500, -75.0, 75.0)
    axg, ayg = O.alpha_grid(pots, grid)
    rng = np.random.default_rng(3003)
    systems = []
    tries = 0
    while len(systems) < N_SYS:
        tries += 1
        zs = rng.uniform(1.0, 6.0)
        f = O.dlsds(inputs.ZL, zs)
        beta = rng.uniform(-15.0, 15.0, 2)
        n, tri, ix, iy = O.find_images(axg, ayg, grid, f, beta[0], beta[1], kmax=32)
        if n < 2 or n > 5:
            continue
        th, res, det = newton(pots, f, beta, np.stack([ix, iy], axis=1))
        if np.max(res) > 1e-10 or np.min(np.abs(det)) < 0.05:
            continue
        if np.max(np.abs(th)) > 70.0:
            continue
        d = np.hypot(th[:, None, 0] - th[None, :, 0], th[:, None, 1] - th[None, :, 1])
        if np.min(d + np.eye(len(th)) * 1e9) < 0.3:
            continue
        systems.append((zs, th))
        print(f"system {len(systems) - 1}: zs={zs:.3f} images={len(th)}", flush=True)
    noise_rng = np.random.default_rng(3004)
    with open(OUT, "w") as fh:
        fh.write("# config-3 constraint catalogue (written by make_cfg3_catalog.py; oracle only)\n")
        fh.write("# model: 300 fixed galaxy dPIEs (seed 3) + 6 free dPIEs at prior midpoints; zl=0.4\n")
        fh.write(f"# {len(systems)} systems, {sum(len(t) for _, t in systems)} images, "
                 f"{tries} sources drawn; noise N(0, {SIGMA}) per coordinate\n")
        fh.write("# columns: system zs x y sigma x_true y_true  [arcsec]\n")
        for i, (zs, th) in enumerate(systems):
            for x, y in th:
                nx_, ny_ = noise_rng.normal(0.0, SIGMA, 2)
                fh.write(f"{i} {zs:.17g} {x + nx_:.17g} {y + ny_:.17g} {SIGMA:.17g} "
                         f"{x:.17g} {y:.17g}\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
