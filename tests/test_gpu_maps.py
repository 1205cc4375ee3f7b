"""GPU parity of the map path (parameter prologue + fused deflection/Hessian
kernel) against the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest

from lensutil import RTOL, assert_within, grid_points

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def phys_to_device(B, phys):
    return B.to_device(phys, B.PHYS_KEYS, "cuda")


def gpu_table(B, ctx, phys):
    return B.table_from_physical(phys_to_device(B, phys), 0, ctx)


def amp_to_device(B, pots):
    return B.to_device(pots, B.POT_KEYS, "cuda")


def run_map(B, ctx, table, grid, dlsds, prec):
    out = B.hessian_map(table, grid, dlsds, prec, with_alpha=True, ctx=ctx)
    torch.cuda.synchronize()
    return np.stack([out[k].double().cpu().numpy() for k in ("ax", "ay", "hxx", "hxy", "hyy")])


def cfg1():
    from paper_2004_06352_amd import inputs
    return inputs.config1()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_config1_full_map(B, ctx, oracle, prec):
    c = cfg1()
    f = oracle.dlsds(c["zl"], c["zs"])
    ref, mag = oracle.lens_map(oracle.phys_to_pots(c["pots"]), c["grid"], f)
    got = run_map(B, ctx, gpu_table(B, ctx, c["pots"]), c["grid"], f, prec)
    worst = assert_within(got, ref, mag, RTOL[prec], f"cfg1 prec={prec}")
    print(f"cfg1 prec={prec} max err/scale = {worst:.3g}")


def test_prologue_matches_oracle_conversion(B, ctx, oracle):
    c = cfg1()
    t = gpu_table(B, ctx, c["pots"])
    o = oracle.phys_to_pots(c["pots"])
    assert np.allclose(t["b0"].cpu().numpy(), o["b0"], rtol=1e-14, atol=0)
    assert np.allclose(t["eps"].cpu().numpy(), o["eps"], rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("shape", [(1, 1), (1, 129), (129, 1), (67, 13), (200, 70), (257, 65)])
def test_ragged_grids(B, ctx, oracle, shape):
    c = cfg1()
    nx, ny = shape
    grid = (nx, ny, -37.3, -81.1, 0.731, 1.377)
    pots = oracle.phys_to_pots(c["pots"])
    ref, mag = oracle.lens_map(pots, grid, 0.6)
    got = run_map(B, ctx, amp_to_device(B, pots), grid, 0.6, 0)
    assert_within(got, ref, mag, RTOL[0], f"grid {shape}")


TUNINGS = [(64, 4, 1, 1, 64), (64, 4, 2, 1, 16), (128, 2, 1, 0, 1), (64, 1, 2, 0, 1),
           (256, 1, 1, 1, 7), (64, 2, 1, 1, 256), (192, 1, 2, 1, 3)]


@pytest.mark.parametrize("tune", TUNINGS)
@pytest.mark.parametrize("prec", [0, 1])
def test_every_launch_configuration(B, oracle, tune, prec):
    c = cfg1()
    ctx = B.Context(0, check=True)
    ctx.set_map_tuning(prec, tune)
    assert ctx.get_map_tuning(prec) == tune
    grid = (131, 37, -50.0, -20.0, 0.77, 1.1)
    pots = oracle.phys_to_pots(c["pots"])
    ref, mag = oracle.lens_map(pots, grid, 0.7)
    got = run_map(B, ctx, amp_to_device(B, pots), grid, 0.7, prec)
    assert_within(got, ref, mag, RTOL[prec], f"tuning {tune}")
    with pytest.raises(B.LensError):
        ctx.set_map_tuning(prec, (65, 4, 1, 1, 64))
    with pytest.raises(B.LensError):
        ctx.set_map_tuning(prec, (64, 8, 1, 1, 64))
    ctx.close()


def special_pots():
    """SIS, cored isothermal ellipsoid without cut, circular dPIE, elliptical
    dPIE with rcore = 0 centred exactly on a grid point, tiny ellipticity."""
    rows = [
        (0.0, 0.0, 10.0, 0.0, 0.0, 0.0, math.inf),        # SIS
        (3.3, -2.1, 6.0, 0.3, 0.7, 0.4, math.inf),        # cored, no cut
        (-5.0, 4.0, 4.0, 0.0, 1.1, 0.5, 30.0),            # circular dPIE
        (1.0, 1.0, 2.0, 0.2, 2.5, 0.0, 15.0),             # singular centre on a grid point
        (7.0, 7.0, 3.0, 1e-10, 0.3, 0.2, 40.0),           # eps -> 0
        (-9.0, -6.0, 0.0, 0.5, 0.0, 0.1, 20.0),           # zero amplitude
    ]
    a = np.array(rows)
    return {k: a[:, i].copy() for i, k in enumerate(("x0", "y0", "b0", "eps", "phi",
                                                     "rcore", "rcut"))}


def test_special_potentials(B, ctx, oracle):
    pots = special_pots()
    grid = (41, 41, -20.0, -20.0, 1.0, 1.0)  # contains (1, 1) and (0, 0) exactly
    ref, mag = oracle.lens_map(pots, grid, 1.0)
    got = run_map(B, ctx, amp_to_device(B, pots), grid, 1.0, 0)
    assert_within(got, ref, mag, RTOL[0], "special potentials")
    for prec in (1, 2):
        got = run_map(B, ctx, amp_to_device(B, pots), grid, 1.0, prec)
        assert_within(got, ref, mag, RTOL[prec], f"special potentials prec={prec}")


def test_fp32_modes_where_single_precision_is_weakest(B, ctx, oracle):
    """Pixels within a few mas of tiny cores 70" from the origin, ellipticity
    1e-7, strong ellipticity, and the far field 1000" away: the FP32 modes keep
    1e-5 of the scale (offsets and rotation are formed in FP64)."""
    rows = [(50.0, -50.0, 0.5, 1e-7, 0.4, 0.005, 10.0),
            (50.01, -49.99, 1.0, 0.45, 2.0, 0.001, 5.0),
            (0.0, 0.0, 40.0, 0.2, 0.5, 5.0, 1000.0)]
    a = np.array(rows)
    pots = {k: a[:, i].copy() for i, k in enumerate(B.POT_KEYS)}
    grids = [(64, 64, 50.0 - 0.0325, -50.0 - 0.0325, 1e-3, 1e-3),
             (48, 40, 49.99, -50.02, 1.7e-3, 1.3e-3),
             (32, 32, 900.0, -1000.0, 1.0, 1.0)]
    for grid in grids:
        ref, mag = oracle.lens_map(pots, grid, 0.8)
        for prec in (1, 2):
            got = run_map(B, ctx, amp_to_device(B, pots), grid, 0.8, prec)
            w = assert_within(got, ref, mag, RTOL[prec], f"fp32 hazard {grid} prec={prec}")
            print(f"hazard grid {grid[:2]} prec={prec}: max err/scale {w:.3g}")


def test_ellipticity_limits_in_every_precision(B, ctx, oracle):
    """Ellipticities around the two switches to the circular closed forms
    (FP64 below 1e-60, FP32 below 1e-8; above them the evaluation divides the
    lengths by k = 2 sqrt(eps)/(1 + eps)), with and without a cut radius: every
    precision, and the FP64 potential map, stay within tolerance of the
    oracle's elliptical forms."""
    rows = []
    for i, e in enumerate((1e-70, 1e-60, 1e-40, 1e-12, 1e-9, 1e-8, 2e-8, 1e-6, 0.3)):
        rows.append((3.0 * i - 12.0, 1.5 * i - 6.0, 2.0 + 0.1 * i, e, 0.37 * i, 0.3, 25.0))
        rows.append((12.0 - 3.0 * i, 1.2 * i - 5.0, 1.5, e, 0.5 + 0.2 * i, 0.4, math.inf))
    a = np.array(rows)
    pots = {k: a[:, i].copy() for i, k in enumerate(B.POT_KEYS)}
    grid = (45, 37, -22.05, -18.05, 1.0, 1.0)
    ref, mag = oracle.lens_map(pots, grid, 0.9)
    for prec in (0, 1, 2):
        got = run_map(B, ctx, amp_to_device(B, pots), grid, 0.9, prec)
        w = assert_within(got, ref, mag, RTOL[prec], f"ellipticity limits prec={prec}")
        print(f"ellipticity limits prec={prec}: max err/scale {w:.3g}")
    pref, pmag = oracle.potential_map(pots, grid, 0.9)
    pgot = B.potential_map(amp_to_device(B, pots), grid, 0.9, ctx=ctx)
    torch.cuda.synchronize()
    assert_within(pgot.cpu().numpy(), pref, pmag, RTOL[0], "ellipticity limits potential")


def test_singular_centre_contributes_zero(B, ctx, oracle):
    one = {k: v[3:4] for k, v in special_pots().items()}
    grid = (3, 3, 0.0, 0.0, 1.0, 1.0)  # (1, 1) is the centre
    got = run_map(B, ctx, amp_to_device(B, one), grid, 1.0, 0)
    assert np.all(got[:, 1, 1] == 0.0)
    assert np.all(np.isfinite(got))


def test_sis_modulus_is_einstein_radius(B, ctx):
    sis = {k: v[0:1] for k, v in special_pots().items()}
    grid = (64, 64, -31.5, -31.5, 1.0, 1.0)  # never hits the centre
    got = run_map(B, ctx, amp_to_device(B, sis), grid, 0.7, 0)
    assert np.allclose(np.hypot(got[0], got[1]), 7.0, rtol=1e-13, atol=0)


def test_empty_table_gives_zero_maps(B, ctx):
    empty = {k: np.zeros(0) for k in B.POT_KEYS}
    got = run_map(B, ctx, amp_to_device(B, empty), (5, 3, 0.0, 0.0, 1.0, 1.0), 1.0, 0)
    assert np.all(got == 0.0)


def test_grad_only_entry_point(B, ctx, oracle):
    c = cfg1()
    pots = oracle.phys_to_pots(c["pots"])
    grid = (100, 50, -60.0, -30.0, 1.2, 1.2)
    ref, mag = oracle.lens_map(pots, grid, 0.7)
    ax, ay = B.grad_map(amp_to_device(B, pots), grid, 0.7, 0, ctx=ctx)
    torch.cuda.synchronize()
    got = np.stack([ax.cpu().numpy(), ay.cpu().numpy()])
    assert_within(got, ref[:2], mag[:2], RTOL[0], "grad only")


def test_config2_full_size_sampled(B, ctx, oracle):
    """2048^2 grid x 502 potentials in FP64 and FP32 evaluation, checked at
    sampled pixels (corners, last row/column, random)."""
    from paper_2004_06352_amd import inputs
    c = inputs.config2()
    f = oracle.dlsds(c["zl"], c["zs"])
    table = gpu_table(B, ctx, c["pots"])
    grid = c["grid"]
    nx, ny = grid[0], grid[1]
    rng = np.random.default_rng(22)
    jj = np.concatenate([[0, 0, ny - 1, ny - 1], rng.integers(0, ny, 1500), np.full(50, ny - 1),
                         rng.integers(0, ny, 50)])
    ii = np.concatenate([[0, nx - 1, 0, nx - 1], rng.integers(0, nx, 1500), rng.integers(0, nx, 50),
                         np.full(50, nx - 1)])
    x, y = grid_points(grid, ii, jj)
    ref, mag = oracle.eval_points(oracle.phys_to_pots(c["pots"]), x, y)
    for prec in (0, 1, 2):
        out = B.hessian_map(table, grid, f, prec, with_alpha=True, ctx=ctx)
        torch.cuda.synchronize()
        got = np.stack([out[k][jj, ii].double().cpu().numpy()
                        for k in ("ax", "ay", "hxx", "hxy", "hyy")])
        del out
        assert_within(got, f * ref, f * mag, RTOL[prec], f"cfg2 sampled prec={prec}")


def test_invalid_table_is_rejected_and_outputs_untouched(B, ctx):
    bad = special_pots()
    bad["eps"][2] = 1.5
    t = B.to_device(bad, B.POT_KEYS, "cuda")
    grid = (8, 8, 0.0, 0.0, 1.0, 1.0)
    out = {k: torch.full((8, 8), 123.0, dtype=torch.float64, device="cuda")
           for k in ("hxx", "hxy", "hyy", "ax", "ay")}
    with pytest.raises(B.LensError) as ei:
        B.hessian_map(t, grid, 1.0, 0, ctx=ctx, out=out)
    assert ei.value.status == -1
    torch.cuda.synchronize()
    for v in out.values():
        assert torch.all(v == 123.0)
    bad = special_pots()
    bad["rcore"][2] = 40.0  # rcore >= rcut
    with pytest.raises(B.LensError):
        B.hessian_map(B.to_device(bad, B.POT_KEYS, "cuda"), grid, 1.0, 0, ctx=ctx)


def test_unchecked_context_reports_invalid_table_later(B):
    ctx = B.Context(0, check=False)
    bad = special_pots()
    bad["b0"][0] = -1.0
    out = B.hessian_map(B.to_device(bad, B.POT_KEYS, "cuda"), (4, 4, 0.5, 0.5, 1.0, 1.0), 1.0,
                        0, ctx=ctx)
    torch.cuda.synchronize()
    assert torch.isnan(out["ax"]).all()
    with pytest.raises(B.LensError):
        ctx.status()
    ctx.status()  # cleared
    ctx.close()


def test_argument_errors(B, ctx):
    t = B.to_device(special_pots(), B.POT_KEYS, "cuda")
    with pytest.raises(B.LensError):
        B.grad_map(t, (0, 4, 0.0, 0.0, 1.0, 1.0), 1.0, 0, ctx=ctx)
    with pytest.raises(B.LensError):
        B.grad_map(t, (4, 4, 0.0, 0.0, 0.0, 1.0), 1.0, 0, ctx=ctx)
    with pytest.raises(B.LensError):
        B.grad_map(t, (4, 4, 0.0, 0.0, 1.0, 1.0), 1.0, 7, ctx=ctx)
    # an output far larger than the allocation it starts in is refused before
    # any launch (a small tensor lives in a 2 MiB segment of torch's allocator)
    small = torch.zeros(3, dtype=torch.float64, device="cuda")
    T, G = B._pot(t), B._grid((8192, 8192, 0.0, 0.0, 1.0, 1.0))
    import ctypes as C
    st = B.lib().lens_grad_map(ctx.handle, C.byref(T), C.byref(G), 1.0, 0, B._ptr(small),
                               B._ptr(small), B._stream())
    assert st == -1
    torch.cuda.synchronize()
    assert torch.all(small == 0)
