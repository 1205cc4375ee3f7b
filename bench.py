"""Benchmark of the lens-gradient hot path on one MI355X.

Primary metric: pixel x potential grad+Hessian evaluations per second of the
fused map kernel on the 2048^2-grid, 502-potential workload (FP64, five output
planes), inputs resident in HBM, each step one lens_hessian_map call (the
parameter prologue and the map kernel).  Secondary metrics in the same JSON
line: FP32-evaluation maps, batched source-plane chi^2 samples/s (4096
samples), the per-sample path on the same batch, the recorded plans
(replayed launches), the sampler, image-plane chi^2 samples/s (eager and
captured in a HIP graph), the
serving streams at 0.7x and 1.5x the plain path's capacity, and, from the
CPU-baseline leg (the oracle timed on the host with all threads and with
one), every map and chi^2 precision's error against the oracle on sampled
pixels and samples.

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
# the same for the deflection alone (the chi^2 kernels): offsets 2, rotation
# 6, per core the radius (q^2 (S^2 + x'^2) + y'^2 and its square root, 5) and
# the two ratios with their arctangent and hyperbolic arctangent (4 + 4), the
# two cores' F (P_a - P_s) 4, rotation back 6, accumulation 2
CHI2_FLOPS_PER_EVAL = 46
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


# ---------------------------------------------------------------------------
# CPU-baseline leg: the oracle timed on the host (all threads, then one), and,
# on the same samples, the GPU results it is set beside compared with it.

def _omp_threads(n):
    """Thread count of the oracle's OpenMP loops (the process's libgomp)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(cpu_model=model, logical_cpus=os.cpu_count(), cpus_available=avail)


def _all_threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def _grow(run, start, total, budget):
    """Run run(n) with n doubling (then scaled to the budget) until one run
    takes about budget seconds or n reaches total -> (n, seconds)."""
    n = start
    while True:
        t0 = time.perf_counter()
        run(n)
        dt = time.perf_counter() - t0
        if dt >= budget or n >= total:
            return n, dt
        n = min(total, max(2 * n, int(n * budget / max(dt, 1e-3) * 1.1)))


def _err_stats(err, scale):
    r = np.abs(err) / np.maximum(scale, 1e-300)
    return {"max_err_over_scale": float(r.max()), "p99_err_over_scale": float(np.percentile(r, 99))}


def cpu_baseline_map(c, f, map_samples, budget_s=12.0, budget_1core_s=6.0):
    """The oracle on a strip of rows of the same map (all potentials), with
    all threads and with one; then the GPU maps of every precision against
    the oracle at the sampled pixels (err / the per-element scale sum_k |term|)."""
    from oracle import oracle as O
    pots = O.phys_to_pots(c["pots"])
    nx, ny, x0, y0, dx, dy = c["grid"]
    npot = len(pots["x0"])

    def run(rows):
        O.lens_map(pots, (nx, rows, x0, y0, dx, dy), f, want_mag=False)

    threads = _all_threads()
    _omp_threads(threads)
    rows, dt = _grow(run, 2, ny, budget_s)
    _omp_threads(1)
    rows1, dt1 = _grow(run, 1, ny, budget_1core_s)
    _omp_threads(threads)
    out = dict(value=nx * rows * npot / dt, unit="pixel*potential evals/s", cores=threads,
               kind="oracle",
               sample=f"{rows} of {ny} rows of the {nx}x{ny} grid, all {npot} potentials, "
                      f"5 channels, {dt:.1f} s",
               value_1core=nx * rows1 * npot / dt1,
               sample_1core=f"{rows1} rows, {dt1:.1f} s", **host_cpu())
    errors = {}
    if map_samples:
        ii, jj = map_samples["ii"], map_samples["jj"]
        # grid points as the grid defines them: one rounded product, one rounded sum
        px = x0 + ii.astype(np.float64) * dx
        py = y0 + jj.astype(np.float64) * dy
        ref, mag = O.eval_points(pots, px, py)
        for name, got in map_samples["values"].items():
            errors[f"map_{name}"] = dict(_err_stats(got - f * ref, f * mag),
                                         points=int(ii.size))
    return out, errors


def _chi2_bound(O, fixed, free, off, cat, m, rtol):
    """Source-plane chi^2 error bound of sample m (unlensed positions each
    within rtol (|theta| + f Sabs))."""
    bx, by, sabs = O.unlens(fixed, free, off, m, cat)
    o = np.asarray(cat["off"])
    total = 0.0
    for i in range(len(o) - 1):
        sl = slice(o[i], o[i + 1])
        if o[i + 1] == o[i]:
            continue
        th = np.hypot(cat["x"][sl], cat["y"][sl])
        e = rtol * (th + cat["f"][i] * sabs[sl])
        D = 2.0 * e.max() + 4e-16 * (th.max() + cat["f"][i] * sabs[sl].max())
        d = np.hypot(bx[sl] - bx[sl].mean(), by[sl] - by[sl].mean())
        total += np.sum((2 * d * D + D * D) / cat["sig"][sl] ** 2)
    return total


def cpu_baseline_chi2(c3, gpu_chi2, budget_s=4.0, budget_1core_s=3.0, n_bound=16):
    """The oracle's source-plane chi^2 (OpenMP over samples) on a prefix of the
    same batch, all threads and one; then the GPU chi^2 of each precision
    against the oracle on that prefix (relative error, and the error over its
    propagated bound on the first n_bound samples)."""
    from oracle import oracle as O
    fixed, free = O.phys_to_pots(c3["fixed"]), O.phys_to_pots(c3["free"])
    cat = O.catalog_f(c3["catalog"], c3["zl"])
    off_all = np.asarray(c3["free_off"])
    total = len(off_all) - 1
    ref = {}

    def run(n):
        ref["chi2"] = O.chi2_source(fixed, free, off_all[:n + 1], cat)

    threads = _all_threads()
    _omp_threads(threads)
    n, dt = _grow(run, 64, total, budget_s)
    ref_chi2 = ref["chi2"]
    _omp_threads(1)
    n1, dt1 = _grow(run, 16, total, budget_1core_s)
    _omp_threads(threads)
    out = dict(value=n / dt, unit="samples/s", cores=threads, kind="oracle",
               sample=f"{n} of the {total} samples, {dt:.1f} s", value_1core=n1 / dt1,
               sample_1core=f"{n1} samples, {dt1:.1f} s")
    errors = {}
    rtol = {"fp64": 1e-12, "fp32_acc64": 1e-5}
    bounds = [_chi2_bound(O, fixed, free, off_all, cat, m, 1.0) for m in range(min(n_bound, n))]
    for name, got in gpu_chi2.items():
        g = np.asarray(got)[:n]
        rel = np.abs(g - ref_chi2) / np.abs(ref_chi2)
        ratio = [abs(g[m] - ref_chi2[m]) / (rtol[name] * bounds[m]) for m in range(len(bounds))]
        errors[f"chi2_source_{name}"] = {"max_rel_err": float(rel.max()),
                                         "max_err_over_bound": float(max(ratio)),
                                         "samples": int(n)}
    return out, errors


def cpu_baseline_image(c4, gpu_img, m1=2):
    """The oracle's image-plane chi^2 of the first m1 samples of the same
    batch (the fixed potentials' vertex deflections computed once, outside
    the timing); then the GPU results of each precision against it: image
    counts that differ, the largest position difference where the counts
    agree, and the chi^2 relative difference."""
    from oracle import oracle as O
    fixed, free = O.phys_to_pots(c4["fixed"]), O.phys_to_pots(c4["free"])
    cat = O.catalog_f(c4["catalog"], c4["zl"])
    grid = c4["grid"]
    threads = _all_threads()
    _omp_threads(threads)
    afix = O.alpha_grid(fixed, grid)
    kmax = next(iter(gpu_img.values()))["img_xy"].shape[2] if gpu_img else 64
    t0 = time.perf_counter()
    ref = O.chi2_image(fixed, free, c4["free_off"], cat, grid, 0, m1, kmax, 100.0,
                       alpha_fix=afix)
    dt = time.perf_counter() - t0
    out = dict(value=m1 / dt, unit="samples/s", cores=threads, kind="oracle",
               sample=f"samples 0..{m1 - 1} of {len(c4['free_off']) - 1} on the "
                      f"{grid[0]}x{grid[1]} grid (fixed part cached), {dt:.1f} s")
    errors = {}
    for name, g in gpu_img.items():
        nimg = g["nimg"][:m1]
        mism = int(np.sum(nimg != ref["nimg"]))
        pos = 0.0
        for m in range(m1):
            for i in range(nimg.shape[1]):
                k = min(int(nimg[m, i]), kmax)
                if nimg[m, i] != ref["nimg"][m, i] or k == 0:
                    continue
                dxy = np.hypot(g["img_xy"][m, i, :k, 0] - ref["x"][m, i, :k],
                               g["img_xy"][m, i, :k, 1] - ref["y"][m, i, :k])
                pos = max(pos, float(dxy.max()))
        rel = np.abs(g["chi2"][:m1] - ref["chi2"]) / np.abs(ref["chi2"])
        errors[f"chi2_image_{name}"] = {"count_mismatches": mism,
                                        "systems": int(nimg.size),
                                        "max_pos_err_arcsec": pos,
                                        "max_chi2_rel_err": float(rel.max()),
                                        "samples": m1}
    return out, errors


def bench_serving(map_rate, chi2_rate, n_requests):
    """Poisson streams of mixed map / chi^2 requests, each served with 4 slots
    and chi^2 merging, then on the plain path (one request at a time, no
    merging).  The arrival rate is a multiple of the plain path's capacity
    estimated from the measured map and chi^2 rates: 0.7 (latency under a
    load the plain path sustains) and 1.5 (saturated: the plain path falls
    behind, so the requests/s each mode completes measure its throughput)."""
    import math

    from paper_2004_06352_amd import inputs, serve
    models = inputs.config5_models()
    sides = (512, 1024, 2048, 4096)
    mean_pix = float(np.mean([s * s for s in sides]))
    mean_npot = float(np.mean([m[0] for m in models]))
    mean_samples = (4096 - 64) / math.log(4096 / 64)
    t_map = mean_pix * mean_npot / map_rate + 2e-4
    t_chi2 = mean_samples / chi2_rate + 2e-4
    capacity = 1.0 / (0.5 * t_map + 0.5 * t_chi2)
    be = serve.GpuBackend(n_slots=4, models=models)
    out = {"workload": f"cfg5_poisson_{n_requests}req", "plain_capacity_est_req_per_s": capacity}
    for load in (0.7, 1.5):
        dicts = inputs.config5_requests(n_requests=n_requests, rate_hz=load * capacity,
                                        map_sides=sides)
        leg = {"rate_hz": load * capacity}
        for name, slots, merge in (("served", 4, True), ("plain", 1, False)):
            reqs = [serve.Req.from_dict(d) for d in dicts]
            be.prepare(reqs)
            st = serve.Scheduler(be, n_slots=slots, merge_chi2=merge).run(reqs)
            leg[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
        leg["served_over_plain_req_per_s"] = leg["served"]["req_per_s"] / leg["plain"]["req_per_s"]
        out[f"load_{load}"] = leg
    return out


def chi2_legs(args, ctx, secondary, torch, B, inputs, keep):
    """Source-plane chi^2 (batched, per-sample, recorded plans), the sampler and
    the image-plane chi^2 (eager and captured); results into `secondary`, the
    GPU outputs the CPU-baseline leg compares with the oracle into `keep`."""
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
    # (enough calls that the closing synchronisation is a small share, after
    # warm-up calls that bring the clock back up; the per-sample path, a long
    # run of one-wave launches that leaves the GPU mostly idle and its clock
    # down, is timed last)
    w, e = timed_steps(lambda: B.chi2_batch(fixed, free, off, cat, ctx=ctx), 200, 20, torch,
                       per_step=False)
    secondary["chi2_source_batched_samples_per_s"] = S * 200 / w
    for name, resident in (("plan", False), ("plan_fixed_resident", True)):
        plan = B.Chi2Plan(fixed, free, off, cat, ctx=ctx, resident=resident)
        w, e = timed_steps(plan.launch, 200, 20, torch, per_step=False)
        secondary[f"chi2_source_{name}_samples_per_s"] = S * 200 / w
        plan.close()
    w, e = timed_steps(lambda: B.chi2_batch(fixed, free, off, cat, path=B.PATH_PER_SAMPLE,
                                            ctx=ctx), 3, 1, torch, per_step=False)
    secondary["chi2_source_per_sample_samples_per_s"] = S * 3 / w
    secondary["chi2_source_workload"] = c3["name"]
    keep["chi2_source"] = {"fp64": B.chi2_batch(fixed, free, off, cat, ctx=ctx)["chi2"].cpu().numpy(),
                           "fp32_acc64": B.chi2_batch(fixed, free, off, cat, prec=B.FP32_ACC64,
                                                      ctx=ctx)["chi2"].cpu().numpy()}
    keep["c3"] = c3
    # Metropolis sampler: 4096 walkers of the same model, one kernel launch
    # per step (proposal, chi^2 and decision per wave); uniforms supplied
    # once and reused (filling them is the caller's generator's cost)
    sm = inputs.sampler_start(n_walkers=4096)
    Wn = sm["params"].shape[0]
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    um = dev(inputs.sampler_uniforms(np.random.default_rng(9), Wn, 6))
    mc = B.Mcmc(fixed, cat, dev(sm["params"]), dev(sm["lo"]), dev(sm["hi"]),
                dev(sm["step"]), um, ctx=ctx)
    w, e = timed_steps(mc.step, 400, 20, torch, per_step=False)
    secondary["mcmc_walker_steps_per_s"] = Wn * 400 / w
    secondary["mcmc_ms_per_step"] = w / 400 * 1e3
    mc.close()
    # the source-plane chi^2 kernel against the FP64 peak, in its sampler
    # form (a step is that one kernel: its launch time is the per-step time
    # on the stream): algorithmic FLOP of a deflection-only evaluation of a
    # two-core dPIE at every (walker, image, free potential)
    nimg = int(c3["catalog"]["off"][-1])
    evals = Wn * nimg * int(sm["params"].shape[1])
    fl = CHI2_FLOPS_PER_EVAL * evals
    secondary["chi2_source_kernel_roofline"] = {
        "kernel": "chi2_src_kernel (sampler form)", "bound": "alu",
        "achieved": fl / e / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
        "frac": fl / e / 1e12 / PEAK_FP64_TFLOPS, "avg_launch_us": e * 1e6,
        "flops_per_eval": CHI2_FLOPS_PER_EVAL, "evals_per_launch": evals}
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
    # the whole image-plane call captured (fixed potentials' vertex
    # deflections and per-image constants kept from creation)
    for name, resident in (("graph", False), ("graph_fixed_resident", True)):
        plan = B.Chi2Plan(fixed, free4, off4, cat, ctx=ctx, resident=resident,
                          mode=B.CHI2_IMAGE, grid=c4["grid"], kmax=64, penalty=100.0)
        w, e = timed_steps(plan.launch, 3, 1, torch, per_step=False)
        secondary[f"chi2_image_fp64_{name}_samples_per_s"] = S4 * 3 / w
        plan.close()
    secondary["chi2_image_workload"] = c4["name"]
    keep["chi2_image"] = {}
    for name, prec in (("fp64", B.FP64), ("fp32_acc64", B.FP32_ACC64)):
        r = B.chi2_batch(fixed, free4, off4, cat, mode=B.CHI2_IMAGE, prec=prec,
                         grid=c4["grid"], kmax=64, penalty=100.0, want_images=True, ctx=ctx)
        keep["chi2_image"][name] = {k: r[k][:2].cpu().numpy() for k in ("chi2", "nimg", "img_xy")}
    keep["c4"] = c4


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
    ap.add_argument("--no-p", action="store_true",
                    help="skip the 5000^2 x 217 deflection map (context leg)")
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
        chi2_legs(args, ctx, secondary, torch, B, inputs, {})
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
        # 64x4 blocks with one pixel per thread, the autotuner's pick here):
        # FP64 vector work actually issued
        rec["roofline"]["executed_flop_per_launch"] = exe
        rec["roofline"]["executed_frac"] = exe / ev / 1e12 / PEAK_FP64_TFLOPS
    secondary = {}
    # pixels at which the CPU-baseline leg compares every map with the oracle
    rs = np.random.default_rng(12)
    ii = rs.integers(0, nx, 2048)
    jj = rs.integers(0, ny, 2048)
    ii_t = torch.as_tensor(ii, device="cuda")
    jj_t = torch.as_tensor(jj, device="cuda")
    chans = ("ax", "ay", "hxx", "hxy", "hyy")

    def gather(o):
        return np.stack([o[k][jj_t, ii_t].double().cpu().numpy() for k in chans])

    map_samples = {"ii": ii, "jj": jj, "values": {"fp64": gather(out)}}
    # FP32 evaluation with FP64 accumulation and compensated FP32
    for name, prec in (("fp32_acc64", B.FP32_ACC64), ("fp32_comp32", B.FP32_COMP32)):
        o32 = {k: torch.empty((ny, nx), dtype=torch.float32, device="cuda") for k in out}
        w32, e32 = timed_steps(lambda: B.hessian_map(table, grid, f, prec, ctx=ctx, out=o32),
                               max(3, args.steps // 2), 1, torch)
        n = max(3, args.steps // 2)
        secondary[f"map_{name}_evals_per_s"] = evals * n / w32
        secondary[f"map_{name}_avg_launch_ms"] = e32 * 1e3
        secondary[f"map_{name}_frac_of_fp32_peak"] = (FLOPS_PER_EVAL * evals / e32 / 1e12 /
                                                      PEAK_FP32_TFLOPS)
        map_samples["values"][name] = gather(o32)
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
    # context: a deflection map of the paper's headline shape (5000^2 grid over
    # 150", 217 potentials), FP64, deflection only as the paper's gradient map
    # (0.93 s on one P100 for its own lens model, Sec. 5)
    if not args.no_p:
        cp = inputs.config_p()
        tp = B.table_from_physical(B.to_device(cp["pots"], B.PHYS_KEYS), 0, ctx)
        npx, npy = cp["grid"][0], cp["grid"][1]
        fp = B.dlsds(cp["zl"], cp["zs"])
        op = {k: torch.empty((npy, npx), dtype=torch.float64, device="cuda") for k in ("ax", "ay")}
        gmap = lambda: B.grad_map(tp, cp["grid"], fp, B.FP64, ctx=ctx, out=op)
        wg, eg = timed_steps(gmap, 5, 2, torch)
        ev_p = npx * npy * int(cp["pots"]["x0"].size)
        secondary["map_P_grad_fp64"] = {"workload": cp["name"], "ms_per_map": eg * 1e3,
                                        "evals_per_s": ev_p / eg,
                                        "paper_single_gpu_s": 0.93,
                                        "paper_single_gpu_evals_per_s": ev_p / 0.93}
        del op, tp
    # lensing potential (FP64), one plane
    op = torch.empty((ny, nx), dtype=torch.float64, device="cuda")
    wp, ep = timed_steps(lambda: B.potential_map(table, grid, f, ctx=ctx, out=op), nd, 1, torch)
    secondary["potential_map_fp64_evals_per_s"] = evals * nd / wp
    secondary["potential_map_fp64_avg_launch_ms"] = ep * 1e3
    del op
    keep = {}
    if not args.no_chi2 and not args.only_map:
        chi2_legs(args, ctx, secondary, torch, B, inputs, keep)
    if not args.no_chi2 and not args.only_map and not args.no_serve:
        log("serving stream")
        secondary["serving"] = bench_serving(value, secondary["chi2_source_batched_samples_per_s"],
                                             args.serve_requests)
    rec["secondary"] = secondary
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        rec["cpu_baseline"], errors = cpu_baseline_map(c2, f, map_samples)
        if "chi2_source" in keep:
            secondary["chi2_source_cpu_baseline"], e2 = cpu_baseline_chi2(keep["c3"],
                                                                       keep["chi2_source"])
            errors.update(e2)
        if "chi2_image" in keep:
            secondary["chi2_image_cpu_baseline"], e3 = cpu_baseline_image(keep["c4"],
                                                                       keep["chi2_image"])
            errors.update(e3)
        secondary["errors_vs_oracle"] = errors
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
