"""The image-plane error bounds of the GPU tests, checked on the CPU with the
oracle alone: every vertex deflection of a lens model is perturbed by up to
rtol times its scale and every source by up to its error bound, the oracle's
brute-force search is run again, and each image must move by no more than
its derived position bound, while any change of an image count or of the
containing triangle must come with the source certified within the error
bound of a triangle edge (Z20, Z21).  The assignment helper is held to the
oracle's own assignment on random systems."""
import math

import numpy as np
import pytest

import lensutil as LU


@pytest.fixture(scope="module")
def lens(oracle):
    from paper_2004_06352_amd import inputs
    fixed = oracle.phys_to_pots(inputs.fixed_galaxies(3))
    free = oracle.phys_to_pots(inputs.truth_free())
    model = {k: np.concatenate([fixed[k], free[k]]) for k in fixed}
    cat = oracle.catalog_f(inputs.load_catalog(), inputs.ZL)
    off = np.array([0, len(free["x0"])], np.int32)
    grid = (161, 161, -32.0, -32.0, 0.4, 0.4)
    ax, ay = oracle.alpha_grid(model, grid)
    _, mag = oracle.lens_map(model, grid, 1.0)
    return dict(fixed=fixed, free=free, model=model, cat=cat, off=off, grid=grid, ax=ax, ay=ay,
                mag=mag)


@pytest.mark.parametrize("rtol", [1e-9, 1e-6, 1e-4])
def test_position_bound_holds_under_perturbed_deflections(oracle, lens, rtol):
    g, cat = lens["grid"], lens["cat"]
    rng = np.random.default_rng(int(-math.log10(rtol)))
    bx, by, sabs = oracle.unlens(lens["fixed"], lens["free"], lens["off"], 0, cat)
    sx, sy = oracle.sources(lens["fixed"], lens["free"], lens["off"], 0, cat)
    serr = LU.source_errors(bx, by, sabs, cat, rtol)
    pax = lens["ax"] + rtol * lens["mag"][0] * rng.uniform(-1, 1, lens["ax"].shape)
    pay = lens["ay"] + rtol * lens["mag"][1] * rng.uniform(-1, 1, lens["ay"].shape)
    scale = float(np.hypot(lens["mag"][0], lens["mag"][1]).max())
    checked = excused = 0
    worst = 0.0
    for i in range(len(sx)):
        f = cat["f"][i]
        n0, t0, x0, y0 = oracle.find_images(lens["ax"], lens["ay"], g, f, sx[i], sy[i], 32)
        t = rng.uniform(0, 2 * math.pi)
        r = serr[i] * rng.uniform(0, 1)
        n1, t1, x1, y1 = oracle.find_images(pax, pay, g, f, sx[i] + r * math.cos(t),
                                            sy[i] + r * math.sin(t), 32)
        if n0 != n1 or not np.array_equal(t0, t1):
            margin = oracle.edge_margin(lens["ax"], lens["ay"], g, f, sx[i], sy[i])
            assert margin <= f * rtol * scale + serr[i] + 64 * LU.U * 100.0, (i, margin)
            excused += 1
            continue
        pos = np.stack([x0, y0], axis=1)
        pb = LU.image_position_bounds(oracle, lens["model"], g, f, serr[i], t0, pos, rtol)
        err = np.hypot(x1 - x0, y1 - y0)
        assert np.all(err <= pb), (i, err, pb)
        checked += len(err)
        if len(err):
            worst = max(worst, float(np.max(err / pb)))
    assert checked >= (100 if rtol < 1e-5 else 20)
    print(f"rtol {rtol:g}: {checked} images within their bounds (largest error/bound "
          f"{worst:.3g}), {excused} systems certified near an edge")


def test_assignment_helper_matches_the_oracle(oracle):
    rng = np.random.default_rng(77)
    for _ in range(300):
        M, n = rng.integers(1, 6), rng.integers(0, 8)
        cx, cy = rng.uniform(-2, 2, M), rng.uniform(-2, 2, M)
        sig = rng.uniform(0.03, 0.1, M)
        ix, iy = rng.uniform(-2.5, 2.5, n), rng.uniform(-2.5, 2.5, n)
        term, miss = LU.system_term(ix, iy, cx, cy, sig, 3.0)
        part, omiss = oracle.assign_system(ix, iy, cx, cy, sig, 3.0)
        assert miss == omiss
        assert term == pytest.approx(part, rel=1e-12, abs=1e-12)


def _as_gpu(ref):
    """The oracle's results in the layout the GPU binding returns."""
    return dict(nimg=ref["nimg"].copy(), chi2=ref["chi2"].copy(), nmissing=ref["nmiss"].copy(),
                img_xy=np.stack([ref["x"], ref["y"]], axis=-1).copy())


def test_comparison_accepts_exact_and_rejects_planted_errors(oracle, lens):
    """compare_image_plane passes the oracle's own results (zero error) and
    fails on a position moved by twice its bound and on an image count
    changed for a system far from every edge."""
    from paper_2004_06352_amd import inputs
    c = inputs.config3(n_samples=2)
    fixed, free = oracle.phys_to_pots(c["fixed"]), oracle.phys_to_pots(c["free"])
    off = np.asarray(c["free_off"])
    cat = lens["cat"]
    g = lens["grid"]
    ref = oracle.chi2_image(fixed, free, off, cat, g, 0, 2, 16, 100.0)
    st = LU.compare_image_plane(oracle, fixed, free, off, cat, g, _as_gpu(ref), ref, [0, 1], 0,
                                1e-12, 100.0)
    assert st["images"] > 50 and st["pos_err"] == 0.0 and st["excused"] == 0
    # one image moved by twice its bound
    s, i = np.argwhere(ref["nimg"] > 0)[0]
    model = {k: np.concatenate([fixed[k], free[k][off[s]:off[s + 1]]]) for k in fixed}
    bx, by, sabs = oracle.unlens(fixed, free, off, s, cat)
    serr = LU.source_errors(bx, by, sabs, cat, 1e-12)
    pos = np.array([[ref["x"][s, i, 0], ref["y"][s, i, 0]]])
    pb = LU.image_position_bounds(oracle, model, g, cat["f"][i], serr[i], ref["tri"][s, i, :1],
                                  pos, 1e-12)[0]
    bad = _as_gpu(ref)
    bad["img_xy"][s, i, 0, 0] += 2 * pb
    with pytest.raises(AssertionError):
        LU.compare_image_plane(oracle, fixed, free, off, cat, g, bad, ref, [0, 1], 0, 1e-12,
                               100.0)
    # one image count changed
    bad = _as_gpu(ref)
    bad["nimg"][s, i] += 1
    with pytest.raises(AssertionError):
        LU.compare_image_plane(oracle, fixed, free, off, cat, g, bad, ref, [0, 1], 0, 1e-12,
                               100.0)
