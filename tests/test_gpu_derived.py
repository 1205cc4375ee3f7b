"""GPU parity of the derived maps (convergence, shear, magnification and the
determinant of the inverse magnification matrix) against the oracle, through
the C ABI: the oracle's derived maps of its own second-derivative map, within
the propagated map tolerance; and the epilogue against the same formulas
applied to the GPU's own second derivatives."""
import numpy as np
import pytest

from lensutil import RTOL, derived_bounds

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NAMES = ("kappa", "gamma1", "gamma2", "gamma", "mu", "det")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_06352_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def ctx(B):
    return B.Context(0, check=True)


def _table(B, ctx, phys):
    return B.table_from_physical(B.to_device(phys, B.PHYS_KEYS, "cuda"), 0, ctx)


def _check(got, ref, bound, what):
    n_mu = 0
    for name in NAMES:
        g = got[name].double().cpu().numpy()
        r, b = ref[name], bound[name]
        use = ~np.isnan(b)
        if name == "mu":
            n_mu = int(use.sum())
        err = np.abs(g - r)
        bad = use & ~(err <= b)
        assert not bad.any(), (f"{what} {name}: {int(bad.sum())} elements out of bound; worst "
                               f"err {err[bad].max():.3g} vs bound {b[bad][np.argmax(err[bad])]:.3g}")
    return n_mu


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_config1_derived_maps(B, ctx, oracle, prec):
    from paper_2004_06352_amd import inputs
    c = inputs.config1()
    f = oracle.dlsds(c["zl"], c["zs"])
    m, mag = oracle.lens_map(oracle.phys_to_pots(c["pots"]), c["grid"], f)
    ref = oracle.derived(m[2], m[3], m[4])
    bound = derived_bounds((m[2], m[3], m[4]), (mag[2], mag[3], mag[4]), RTOL[prec], prec != 0)
    got = B.derived_map(_table(B, ctx, c["pots"]), c["grid"], f, prec, ctx=ctx)
    torch.cuda.synchronize()
    n_mu = _check(got, ref, bound, f"cfg1 prec={prec}")
    crit = int((np.sign(ref["det"][:, 1:]) != np.sign(ref["det"][:, :-1])).sum())
    print(f"cfg1 prec={prec}: mu compared at {n_mu} of {ref['mu'].size} pixels; "
          f"{crit} critical-line crossings along rows")
    assert crit > 0  # the field holds critical lines, where mu changes sign


@pytest.mark.parametrize("shape,tune", [((67, 13), (64, 4, 1, 1, 64)), ((300, 170), (64, 4, 2, 1, 16)),
                                        ((129, 1), (128, 2, 1, 0, 1)), ((1, 129), (256, 1, 2, 1, 7))])
def test_derived_epilogue_matches_formulas_on_gpu_hessian(B, oracle, shape, tune):
    """Same launch shape, same accumulated sums: the epilogue's outputs are
    the stated formulas of the GPU's own second derivatives (bit for bit;
    the square root and the reciprocal are correctly rounded on both sides)."""
    from paper_2004_06352_amd import inputs
    ctx = B.Context(0, check=False)
    ctx.set_map_tuning(B.FP64, tune)
    c = inputs.config1()
    nx, ny = shape
    grid = (nx, ny, -37.3, -81.1, 0.731, 1.377)
    t = _table(B, ctx, c["pots"])
    h = B.hessian_map(t, grid, 0.7, B.FP64, with_alpha=False, ctx=ctx)
    got = B.derived_map(t, grid, 0.7, B.FP64, ctx=ctx)
    torch.cuda.synchronize()
    hxx, hxy, hyy = (h[k].cpu().numpy() for k in ("hxx", "hxy", "hyy"))
    k = 0.5 * (hxx + hyy)
    g1 = 0.5 * (hxx - hyy)
    gg = g1 * g1 + hxy * hxy
    det = (1.0 - k) * (1.0 - k) - gg
    with np.errstate(divide="ignore"):
        want = dict(kappa=k, gamma1=g1, gamma2=hxy, gamma=np.sqrt(gg), mu=1.0 / det, det=det)
    for name in NAMES:
        assert np.array_equal(got[name].cpu().numpy(), want[name]), name
    ctx.close()


def test_derived_outputs_subset_and_errors(B, ctx):
    from paper_2004_06352_amd import inputs
    c = inputs.config1()
    t = _table(B, ctx, c["pots"])
    grid = (50, 40, -10.0, -8.0, 0.4, 0.4)
    full = B.derived_map(t, grid, 0.7, B.FP64, ctx=ctx)
    part = B.derived_map(t, grid, 0.7, B.FP64, names=("mu",), ctx=ctx)
    torch.cuda.synchronize()
    assert set(part) == {"mu"} and torch.equal(part["mu"], full["mu"])
    with pytest.raises(B.LensError):
        B.derived_map(t, grid, 0.7, B.FP64, names=(), ctx=ctx)
    with pytest.raises(B.LensError):  # output far smaller than the grid: refused before launch
        B.derived_map(t, (8192, 8192, 0.0, 0.0, 0.01, 0.01), 0.7, B.FP64, ctx=ctx,
                      out={"kappa": torch.empty(10, dtype=torch.float64, device="cuda")})


def test_config2_full_size_sampled(B, ctx, oracle):
    """Derived maps of the 2048^2 x 502 workload (FP64, the benchmark's
    model) at 1200 sampled pixels (corners and random) against the oracle's
    formulas applied to its own second derivatives there."""
    from lensutil import grid_points
    from paper_2004_06352_amd import inputs
    c = inputs.config2()
    f = oracle.dlsds(c["zl"], c["zs"])
    grid = c["grid"]
    nx, ny = grid[0], grid[1]
    rng = np.random.default_rng(31)
    jj = np.concatenate([[0, 0, ny - 1, ny - 1], rng.integers(0, ny, 1196)])
    ii = np.concatenate([[0, nx - 1, 0, nx - 1], rng.integers(0, nx, 1196)])
    x, y = grid_points(grid, ii, jj)
    val, mag = oracle.eval_points(oracle.phys_to_pots(c["pots"]), x, y)
    h = (f * val[2], f * val[3], f * val[4])
    ref = oracle.derived(*h)
    bound = derived_bounds(h, (f * mag[2], f * mag[3], f * mag[4]), RTOL[0])
    got = B.derived_map(_table(B, ctx, c["pots"]), grid, f, 0, ctx=ctx)
    torch.cuda.synchronize()
    sampled = {k: v[jj, ii] for k, v in got.items()}
    n_mu = _check(sampled, ref, bound, "cfg2 sampled")
    print(f"cfg2 derived sampled: mu compared at {n_mu} of {len(ii)} pixels")
