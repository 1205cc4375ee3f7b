"""The map autotuner: every candidate launch configuration gives bit-identical
maps (launch shape never changes what is summed or in which order), and the
chosen configuration is installed in the context."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_tuner_candidates_are_bit_identical(prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_06352_amd import binding as B
    from paper_2004_06352_amd import inputs, tune
    c = inputs.config1()
    ctx = B.Context(0, check=False)
    table = B.table_from_physical(B.to_device(c["pots"], B.PHYS_KEYS), 0, ctx)
    grid = (300, 170, -100.0, -60.0, 0.66, 0.7)
    best, results = tune.tune_map(ctx, table, grid, prec, reps=1, use_cache=False)
    assert len(results) == len(tune.candidates()), "some launch shape changed the output"
    assert ctx.get_map_tuning(prec) == tuple(best)
    assert results[0][1] <= results[-1][1]
    ctx.close()


def test_chi2_tuner_choices_are_bit_identical():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_06352_amd import binding as B
    from paper_2004_06352_amd import inputs, tune
    c = inputs.config3(n_samples=700, uneven=True)
    ctx = B.Context(0, check=False)
    fixed = B.table_from_physical(B.to_device(c["fixed"], B.PHYS_KEYS), 0, ctx)
    free = B.table_from_physical(B.to_device(c["free"], B.PHYS_KEYS), 0, ctx)
    off = torch.as_tensor(c["free_off"], dtype=torch.int32, device="cuda")
    cat = B.catalog_to_device(B.catalog_with_dlsds(c["catalog"], c["zl"]))
    best, results = tune.tune_chi2(ctx, fixed, free, off, cat, reps=1)
    assert len(results) == 6 and ctx.get_chi2_tuning() == best
    with pytest.raises(B.LensError):
        ctx.set_chi2_tuning(0)
    ctx.close()
