"""The allocation-free map call (lens_hessian_map_noalloc) against
lens_hessian_map, through the C ABI: two calls in a row, the second on a
smaller table and grid, each bit-identical to the allocating call on the same
inputs and launch shape (both run the same prologue and map kernels), and
still within the FP64 tolerance of the oracle."""
import numpy as np
import pytest

from lensutil import RTOL, assert_within

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PLANES = ("ax", "ay", "hxx", "hxy", "hyy")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_06352_amd import binding
    binding.lib()
    return binding


def _planes(nx, ny, dtype):
    return {k: torch.full((ny, nx), float("nan"), dtype=dtype, device="cuda") for k in PLANES}


def _np(out):
    return np.stack([out[k].double().cpu().numpy() for k in PLANES])


def _case(inputs, n_pot, side):
    """Cfg-2 style table (2 cluster halos + galaxies) of n_pot potentials on a
    side x side grid over 200 arcsec."""
    c = inputs.config2(n=side, n_gal=n_pot - 2)
    return c


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_allocating_call_twice(B, oracle, prec):
    from paper_2004_06352_amd import inputs
    ctx = B.Context(0, check=True)
    dt = torch.float64 if prec == 0 else torch.float32
    for n_pot, side in ((700, 200), (90, 131)):
        c = _case(inputs, n_pot, side)
        f = B.dlsds(c["zl"], c["zs"])
        table = B.table_from_physical(B.to_device(c["pots"], B.PHYS_KEYS), 0, ctx)
        nx, ny = c["grid"][0], c["grid"][1]
        ref_out = _planes(nx, ny, dt)
        B.hessian_map(table, c["grid"], f, prec, ctx=ctx, out=ref_out)
        got_out = _planes(nx, ny, dt)
        B.hessian_map_noalloc(table, c["grid"], f, prec, ctx=ctx, out=got_out)
        torch.cuda.synchronize()
        ref, got = _np(ref_out), _np(got_out)
        assert np.isfinite(got).all(), f"n_pot={n_pot}: unwritten or NaN output"
        assert np.array_equal(got.view(np.int64), ref.view(np.int64)), \
            f"n_pot={n_pot} side={side} prec={prec}: not bit-identical to lens_hessian_map"
        # and both within the tolerance of the oracle on a strip of rows
        rows = (0, 3)
        g = c["grid"]
        strip = (nx, rows[1] - rows[0], g[2], g[3] + rows[0] * g[5], g[4], g[5])
        o_ref, o_mag = oracle.lens_map(oracle.phys_to_pots(c["pots"]), strip,
                                       oracle.dlsds(c["zl"], c["zs"]))
        worst = assert_within(got[:, rows[0]:rows[1], :], o_ref, o_mag, RTOL[prec],
                              f"noalloc n_pot={n_pot} prec={prec}")
        print(f"noalloc n_pot={n_pot} side={side} prec={prec}: bit-identical, "
              f"max err/scale vs oracle {worst:.3g}")
    ctx.close()


def test_noalloc_rejects_a_table_beyond_its_limit(B):
    from paper_2004_06352_amd import inputs
    ctx = B.Context(0, check=True)
    c = inputs.config2(n=64, n_gal=B.NOALLOC_MAX_POT + 1 - 2)
    table = B.table_from_physical(B.to_device(c["pots"], B.PHYS_KEYS), 0, ctx)
    out = _planes(64, 64, torch.float64)
    with pytest.raises(B.LensError) as ei:
        B.hessian_map_noalloc(table, c["grid"], 0.7, 0, ctx=ctx, out=out)
    assert ei.value.status == -2
    torch.cuda.synchronize()
    assert torch.isnan(out["hxx"]).all(), "a rejected call wrote its output"
    ctx.close()
