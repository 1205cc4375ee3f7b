"""Benchmark of the lens-gradient hot path on one MI355X.

Primary metric: pixel x potential grad+Hessian evaluations per second of the
fused map kernel on the 2048^2-grid, 502-potential workload (FP64, five output
planes), inputs resident in HBM, each step one lens_hessian_map call (the
parameter prologue and the map kernel).  Secondary metrics in the same JSON
line: FP32-evaluation maps, batched source-plane chi^2 samples/s (4096
samples), the per-sample path on the same batch, the captured (HIP graph)
batch, and image-plane chi^2 samples/s.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-chi2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic FP64 operations per (pixel, potential) evaluation of an
# elliptical two-core dPIE with deflection and second derivatives, counted
# from the closed forms (each +, -, *, /, sqrt, atan, atanh = 1)
FLOPS_PER_EVAL = 103
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(fn, steps, warmup, torch, per_step=True):
    """Wall time of `steps` calls of fn and the mean per-call time on the
    current stream from HIP events.  per_step=False brackets the whole loop
    with one pair of events: an event record between calls costs ~17 us of
    device time here, which would dominate calls of ~70 us."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if not per_step:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, e0.elapsed_time(e1) * 1e-3 / steps
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record()
        fn()
        ends[k].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = [s.elapsed_time(e) * 1e-3 for s, e in zip(starts, ends)]
    return wall, float(np.mean(ev))


MAP_SOURCES = ("paper_2004_06352_amd/csrc/maps.hip", "paper_2004_06352_amd/csrc/eval.h",
               "paper_2004_06352_amd/csrc/lens_internal.h",
               "paper_2004_06352_amd/csrc/series_coeffs.h",
               "paper_2004_06352_amd/csrc/prologue.h")
COUNTERS = os.path.join(ROOT, "profiles", "map_kernel_cfg2_2048sq_502pot_counters.md")


def map_source_hash():
    """Hash of the code (comments and blank lines dropped) of the sources that
    define the map kernel."""
    import hashlib
    import re
    h = hashlib.sha256()
    for p in MAP_SOURCES:
        with open(os.path.join(ROOT, p)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.split("\n"):
            line = line.split("//", 1)[0].strip()
            if line:
                h.update(line.encode() + b"\n")
    return h.hexdigest()[:16]


def _counters():
    """key: value lines of the committed counter summary, or None when the
    counters were taken on other kernel sources."""
    if not os.path.exists(COUNTERS):
        return None
    kv = {}
    with open(COUNTERS) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != map_source_hash():
        return None
    return kv


def measured_executed_flop():
    """Executed FP64 FLOP per map launch (64 (ADD + MUL + TRANS) + 128 FMA per
    wave instruction, from the committed VALU counter pass), or None."""
    kv = _counters()
    if kv is None or "map_executed_flop" not in kv:
        return None
    return float(kv["map_executed_flop"])


def measured_traffic():
    """HBM bytes per FP64 map launch from the committed FETCH_SIZE / WRITE_SIZE
    passes, each scaled by what the same counter read for a plain copy of known
    size; None when the counters were taken on other kernel sources."""
    kv = _counters()
    if kv is None:
        return None
    copy_bytes = float(kv["copy_bytes"])
    fetch = float(kv["map_fetch_kib"]) * copy_bytes / (1024 * float(kv["copy_fetch_kib"]))
    write = float(kv["map_write_kib"]) * copy_bytes / (1024 * float(kv["copy_write_kib"]))
    return (fetch + write) * 1024


def cpu_baseline_map(c, budget_s=12.0):
    """The oracle on a strip of rows of the same map (all potentials)."""
    from oracle import oracle as O
    pots = O.phys_to_pots(c["pots"])
    f = O.dlsds(c["zl"], c["zs"])
    nx, ny, x0, y0, dx, dy = c["grid"]
    npot = len(pots["x0"])
    rows = 2
    while True:
        g = (nx, rows, x0, y0, dx, dy)
        t0 = time.perf_counter()
        O.lens_map(pots, g, f, want_mag=False)
        dt = time.perf_counter() - t0
        if dt >= budget_s or rows >= ny:
            break
        rows = min(ny, max(rows * 2, int(rows * budget_s / max(dt, 1e-3) * 1.1)))
    evals = nx * rows * npot
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=evals / dt, unit="pixel*potential evals/s", cores=threads, kind="oracle",
                sample=f"{rows} of {ny} rows of the {nx}x{ny} grid, all {npot} potentials, "
                       f"5 channels, {dt:.1f} s")


def cpu_baseline_chi2(c3, budget_s=4.0):
    """The oracle's source-plane chi^2 (OpenMP over samples) on a prefix of the
    same batch, grown until it takes about budget_s."""
    from oracle import oracle as O
    fixed, free = O.phys_to_pots(c3["fixed"]), O.phys_to_pots(c3["free"])
    cat = O.catalog_f(c3["catalog"], c3["zl"])
    off_all = np.asarray(c3["free_off"])
    total = len(off_all) - 1
    n = 64
    while True:
        off = off_all[:n + 1]
        t0 = time.perf_counter()
        O.chi2_source(fixed, free, off, cat)
        dt = time.perf_counter() - t0
        if dt >= budget_s or n >= total:
            break
        n = min(total, max(2 * n, int(n * budget_s / max(dt, 1e-3) * 1.1)))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=n / dt, unit="samples/s", cores=threads, kind="oracle",
                sample=f"{n} of the {total} samples, {dt:.1f} s")


def bench_serving(map_rate, chi2_rate, n_requests):
    """Poisson stream of mixed map / chi^2 requests at 0.7x the single-stream
    capacity estimated from the measured map and chi^2 rates; served with 4
    slots and chi^2 merging, then the same stream on the plain path (one
    request at a time, no merging)."""
    import math

    from paper_2004_06352_amd import inputs, serve
    models = inputs.config5_models()
    sides = (512, 1024, 2048, 4096)
    mean_pix = float(np.mean([s * s for s in sides]))
    mean_npot = float(np.mean([m[0] for m in models]))
    mean_samples = (4096 - 64) / math.log(4096 / 64)
    t_map = mean_pix * mean_npot / map_rate + 2e-4
    t_chi2 = mean_samples / chi2_rate + 2e-4
    rate = 0.7 / (0.5 * t_map + 0.5 * t_chi2)
    dicts = inputs.config5_requests(n_requests=n_requests, rate_hz=rate, map_sides=sides)
    be = serve.GpuBackend(n_slots=4, models=models)
    out = {"workload": f"cfg5_poisson_{n_requests}req", "rate_hz": rate}
    for name, slots, merge in (("served", 4, True), ("plain", 1, False)):
        reqs = [serve.Req.from_dict(d) for d in dicts]
        be.prepare(reqs)
        st = serve.Scheduler(be, n_slots=slots, merge_chi2=merge).run(reqs)
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
    return out


def chi2_legs(args, ctx, secondary, torch, B, inputs):
    """Source-plane chi^2 (batched, per-sample, graph plans), the sampler and
    the image-plane chi^2; results into `secondary`."""
    c3 = inputs.config3()
    cat = B.catalog_to_device(B.catalog_with_dlsds(c3["catalog"], c3["zl"]))
    fixed = B.table_from_physical(B.to_device(c3["fixed"], B.PHYS_KEYS), 0, ctx)
    free = B.table_from_physical(B.to_device(c3["free"], B.PHYS_KEYS), 0, ctx)
    off = torch.as_tensor(c3["free_off"], dtype=torch.int32, device="cuda")
    S = int(off.numel()) - 1
    if not args.no_tune:
        from paper_2004_06352_amd import tune
        wpc, _ = tune.tune_chi2(ctx, fixed, free, off, cat)
        secondary["chi2_source_waves_per_cu"] = wpc
    for name, path in (("batched", B.PATH_BATCHED), ("per_sample", B.PATH_PER_SAMPLE)):
        n = 50 if path == B.PATH_BATCHED else 3
        w, e = timed_steps(lambda: B.chi2_batch(fixed, free, off, cat, path=path, ctx=ctx),
                           n, 1, torch, per_step=False)
        secondary[f"chi2_source_{name}_samples_per_s"] = S * n / w
    for name, resident in (("graph", False), ("graph_fixed_resident", True)):
        plan = B.Chi2Plan(fixed, free, off, cat, ctx=ctx, resident=resident)
        w, e = timed_steps(plan.launch, 50, 2, torch, per_step=False)
        secondary[f"chi2_source_{name}_samples_per_s"] = S * 50 / w
        plan.close()
    secondary["chi2_source_workload"] = c3["name"]
    if not args.no_cpu:
        secondary["chi2_source_cpu_baseline"] = cpu_baseline_chi2(c3)
    # Metropolis sampler: 4096 walkers of the same model, one kernel launch
    # per step (proposal, chi^2 and decision per wave); uniforms supplied
    # once and reused (filling them is the caller's generator's cost)
    sm = inputs.sampler_start(n_walkers=4096)
    Wn = sm["params"].shape[0]
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    um = dev(inputs.sampler_uniforms(np.random.default_rng(9), Wn, 6))
    mc = B.Mcmc(fixed, cat, dev(sm["params"]), dev(sm["lo"]), dev(sm["hi"]),
                dev(sm["step"]), um, ctx=ctx)
    w, e = timed_steps(mc.step, 100, 3, torch, per_step=False)
    secondary["mcmc_walker_steps_per_s"] = Wn * 100 / w
    secondary["mcmc_ms_per_step"] = w / 100 * 1e3
    mc.close()
    if args.no_image:
        return
    # image-plane chi^2: 1000^2 grid, 512 samples of the same model
    c4 = inputs.config4()
    off4 = torch.as_tensor(c4["free_off"], dtype=torch.int32, device="cuda")
    free4 = B.table_from_physical(B.to_device(c4["free"], B.PHYS_KEYS), 0, ctx)
    S4 = int(off4.numel()) - 1
    for name, prec in (("fp64", B.FP64), ("fp32_acc64", B.FP32_ACC64)):
        w, e = timed_steps(lambda: B.chi2_batch(fixed, free4, off4, cat, mode=B.CHI2_IMAGE,
                                                prec=prec, grid=c4["grid"], kmax=64,
                                                penalty=100.0, ctx=ctx), 3, 1, torch,
                           per_step=False)
        secondary[f"chi2_image_{name}_samples_per_s"] = S4 * 3 / w
    # the same with every found image refined by Newton's method to 1e-10"
    w, e = timed_steps(lambda: B.chi2_batch(fixed, free4, off4, cat, mode=B.CHI2_IMAGE,
                                            grid=c4["grid"], kmax=64, penalty=100.0,
                                            refine=(20, 1e-10), ctx=ctx), 3, 1, torch,
                       per_step=False)
    secondary["chi2_image_fp64_refined_samples_per_s"] = S4 * 3 / w
    secondary["chi2_image_workload"] = c4["name"]


def chi2_source_only(args, ctx, torch, B, inputs):
    """Profiling aid: the batched source-plane chi^2 call and the sampler step
    on the workload-3 batch, `args.steps` of each after one warm-up."""
    c3 = inputs.config3()
    cat = B.catalog_to_device(B.catalog_with_dlsds(c3["catalog"], c3["zl"]))
    fixed = B.table_from_physical(B.to_device(c3["fixed"], B.PHYS_KEYS), 0, ctx)
    free = B.table_from_physical(B.to_device(c3["free"], B.PHYS_KEYS), 0, ctx)
    off = torch.as_tensor(c3["free_off"], dtype=torch.int32, device="cuda")
    S = int(off.numel()) - 1
    w, e = timed_steps(lambda: B.chi2_batch(fixed, free, off, cat, ctx=ctx), args.steps, 1,
                       torch, per_step=False)
    sm = inputs.sampler_start(n_walkers=4096)
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    um = dev(inputs.sampler_uniforms(np.random.default_rng(9), sm["params"].shape[0], 6))
    mc = B.Mcmc(fixed, cat, dev(sm["params"]), dev(sm["lo"]), dev(sm["hi"]), dev(sm["step"]),
                um, ctx=ctx)
    wm, em = timed_steps(mc.step, args.steps, 1, torch, per_step=False)
    mc.close()
    log(json.dumps({"chi2_source_batched_us_per_call": e * 1e6,
                    "chi2_source_batched_samples_per_s": S / e,
                    "mcmc_us_per_step": em * 1e6}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-chi2", action="store_true")
    ap.add_argument("--only-map", action="store_true", help="primary map metric only")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--launch", default="", help="fixed FP64 map launch bx,by,ppt,stage,chunk")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--skip-map", action="store_true",
                    help="profiling aid: no map timing; the chi^2 legs only (no JSON line)")
    ap.add_argument("--no-image", action="store_true", help="skip the image-plane chi^2 legs")
    ap.add_argument("--only-chi2-source", action="store_true",
                    help="profiling aid: `--steps` batched source-plane chi^2 calls on the "
                         "4096-sample batch and as many sampler steps, nothing else")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library has no "
              "multi-GPU path (maps would shard by pixel bands and chi^2 batches by sample).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2004_06352_amd import binding as B
    from paper_2004_06352_amd import inputs

    torch.cuda.set_device(0)
    ctx = B.Context(0, check=False)
    if args.only_chi2_source:
        chi2_source_only(args, ctx, torch, B, inputs)
        return
    c2 = inputs.config2()
    f = B.dlsds(c2["zl"], c2["zs"])
    phys = B.to_device(c2["pots"], B.PHYS_KEYS)
    table = B.table_from_physical(phys, 0, ctx)
    grid = c2["grid"]
    nx, ny, npot = grid[0], grid[1], int(c2["pots"]["x0"].size)
    out = {k: torch.empty((ny, nx), dtype=torch.float64, device="cuda")
           for k in ("hxx", "hxy", "hyy", "ax", "ay")}

    def step():
        B.hessian_map(table, grid, f, B.FP64, ctx=ctx, out=out)

    if args.copy_probe_mib:
        # a plain device copy of known size: the reference the HBM byte
        # counters of the map kernel are scaled by
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tuned = {}
    if args.launch:
        ctx.set_map_tuning(B.FP64, tuple(int(v) for v in args.launch.split(",")))
    elif not args.no_tune:
        from paper_2004_06352_amd import tune
        for prec in (B.FP64, B.FP32_ACC64, B.FP32_COMP32):
            best, _ = tune.tune_map(ctx, table, grid, prec, reps=2)
            tuned[prec] = list(best)
        log(f"tuned launch shapes: {tuned}")
    if args.skip_map:
        secondary = {}
        chi2_legs(args, ctx, secondary, torch, B, inputs)
        log(json.dumps(secondary))
        return
    log(f"map {nx}x{ny} x {npot} potentials, FP64, steps={args.steps}")
    wall, ev = timed_steps(step, args.steps, args.warmup, torch)
    evals = nx * ny * npot
    value = evals * args.steps / wall
    ms = wall / args.steps * 1e3
    achieved = FLOPS_PER_EVAL * evals / ev / 1e12
    rec = {
        "metric": "pixel*potential grad+Hessian evals/s",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": c2["name"], "grid": [nx, ny], "potentials": npot,
                   "channels": 5, "precision": "fp64",
                   "launch": ctx.get_map_tuning(B.FP64)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic(), "traffic_unit": "bytes per launch",
                     "algorithmic_bytes": 5 * 8 * nx * ny,
                     "kernel": "map_kernel<fp64, grad+hess>", "flops_per_eval": FLOPS_PER_EVAL,
                     "avg_launch_ms": ev * 1e3},
    }
    exe = measured_executed_flop()
    if exe is not None:
        # the executed-instruction view of the same launches (counters taken on
        # 64x4 blocks with two pixels per thread, the autotuner's pick here):
        # FP64 vector work actually issued
        rec["roofline"]["executed_flop_per_launch"] = exe
        rec["roofline"]["executed_frac"] = exe / ev / 1e12 / PEAK_FP64_TFLOPS
    secondary = {}
    # FP32 evaluation with FP64 accumulation and compensated FP32
    for name, prec in (("fp32_acc64", B.FP32_ACC64), ("fp32_comp32", B.FP32_COMP32)):
        o32 = {k: torch.empty((ny, nx), dtype=torch.float32, device="cuda") for k in out}
        w32, e32 = timed_steps(lambda: B.hessian_map(table, grid, f, prec, ctx=ctx, out=o32),
                               max(3, args.steps // 2), 1, torch)
        n = max(3, args.steps // 2)
        secondary[f"map_{name}_evals_per_s"] = evals * n / w32
        secondary[f"map_{name}_avg_launch_ms"] = e32 * 1e3
        del o32
    # derived maps (convergence, shear, magnification, det) in FP64: second
    # derivatives only, with the derived epilogue; six planes written
    od = {k: torch.empty((ny, nx), dtype=torch.float64, device="cuda") for k in B.DERIVED}
    nd = max(3, args.steps // 2)
    wd, ed = timed_steps(lambda: B.derived_map(table, grid, f, B.FP64, ctx=ctx, out=od), nd, 1,
                         torch)
    secondary["derived_map_fp64_evals_per_s"] = evals * nd / wd
    secondary["derived_map_fp64_avg_launch_ms"] = ed * 1e3
    del od
    # lensing potential (FP64), one plane
    op = torch.empty((ny, nx), dtype=torch.float64, device="cuda")
    wp, ep = timed_steps(lambda: B.potential_map(table, grid, f, ctx=ctx, out=op), nd, 1, torch)
    secondary["potential_map_fp64_evals_per_s"] = evals * nd / wp
    secondary["potential_map_fp64_avg_launch_ms"] = ep * 1e3
    del op
    if not args.no_chi2 and not args.only_map:
        chi2_legs(args, ctx, secondary, torch, B, inputs)
    if not args.no_chi2 and not args.only_map and not args.no_serve:
        log("serving stream")
        secondary["serving"] = bench_serving(value, secondary["chi2_source_batched_samples_per_s"],
                                             args.serve_requests)
    rec["secondary"] = secondary
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        rec["cpu_baseline"] = cpu_baseline_map(c2)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
