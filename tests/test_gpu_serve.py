"""Serving on the GPU: every result of a mixed, overlapped, merged request
stream is bit-identical to the same request served alone; a map result is
checked against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def serve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_06352_amd import binding, serve
    binding.lib()
    return serve


def small_stream(inputs, n=48):
    kw = dict(map_sides=(128, 256, 384), n_models=4, pot_range=(20, 120),
              batch_range=(16, 300))
    reqs = inputs.config5_requests(seed=7, n_requests=n, rate_hz=400.0, **kw)
    models = inputs.config5_models(7, kw["n_models"], kw["pot_range"])
    return reqs, models


def test_mixed_stream_equals_alone(serve, oracle):
    from paper_2004_06352_amd import inputs
    dicts, models = small_stream(inputs)
    be = serve.GpuBackend(n_slots=4, models=models)
    mix = [serve.Req.from_dict(d) for d in dicts]
    be.prepare(mix)
    st = serve.Scheduler(be, n_slots=4, keep_results=True).run(mix)
    torch.cuda.synchronize()
    assert st["requests"] == len(mix)
    print("mix stats:", {k: round(v, 3) if isinstance(v, float) else v for k, v in st.items()})
    for r in mix:
        alone = serve.Req.from_dict(dict(dicts[r.id], t=0.0))
        serve.Scheduler(be, n_slots=1, merge_chi2=False, keep_results=True).run([alone])
        torch.cuda.synchronize()
        if r.kind == "map":
            for k in ("ax", "ay", "hxx", "hxy", "hyy"):
                assert torch.equal(r.result[k], alone.result[k]), (r.id, k)
        else:
            assert torch.equal(r.result, alone.result), r.id
    # one map result against the oracle at sampled pixels
    r = next(x for x in mix if x.kind == "map")
    pots = oracle.phys_to_pots(inputs.map_request_pots(r.npot, r.model_seed))
    grid = be.grid(r.side)
    f = oracle.dlsds(inputs.ZL, 2.0)
    rng = np.random.default_rng(1)
    ii, jj = rng.integers(0, r.side, 200), rng.integers(0, r.side, 200)
    x, y = grid[2] + ii * grid[4], grid[3] + jj * grid[5]
    ref, mag = oracle.eval_points(pots, x, y)
    got = np.stack([r.result[k][jj, ii].cpu().numpy() for k in ("ax", "ay", "hxx", "hxy", "hyy")])
    assert np.all(np.abs(got - f * ref) <= 1e-12 * f * mag)


def test_budget_defers_on_the_device(serve):
    from paper_2004_06352_amd import inputs
    dicts, models = small_stream(inputs, n=24)
    be = serve.GpuBackend(n_slots=4, models=models)
    reqs = [serve.Req.from_dict(dict(d, t=0.0)) for d in dicts]
    be.prepare(reqs)
    big = max(be.footprint([r]) for r in reqs)
    st = serve.Scheduler(be, n_slots=4, hbm_budget=int(1.5 * big)).run(reqs)
    assert st["deferred"] >= 1 and st["peak_bytes"] <= int(1.5 * big)
