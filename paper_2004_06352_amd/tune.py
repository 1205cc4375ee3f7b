"""Autotuner for the map kernel's launch configuration.

For a given workload (potential table, grid, precision) it times every
candidate (block shape, points per thread, LDS staging or wave-uniform loads,
LDS chunk) with HIP events on the current stream, keeps the fastest whose
output is bit-identical to the default configuration's (a launch shape never
changes what is summed or in which order, so it must never change a bit), and
installs it in the library context.  Results are cached per (device, precision,
output mode, size class) in a JSON file next to the built library.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import binding as B

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_native", "map_tuning.json")

DEFAULT = (64, 4, 2, 1, 64)


def candidates():
    out = []
    for bx, by in ((64, 1), (64, 2), (64, 4), (128, 1), (128, 2), (256, 1)):
        for ppt in (1, 2):
            out.append((bx, by, ppt, 0, 1))
            for chunk in (32, 64, 128):
                out.append((bx, by, ppt, 1, chunk))
    return out


def size_class(grid, npot):
    """Bucket workloads so that one tuning serves similar shapes."""
    pix = int(grid[0]) * int(grid[1])
    return f"pix{max(0, pix.bit_length() - 1)}_pot{max(0, int(npot).bit_length() - 1)}"


def _key(prec, hess, grid, npot):
    name = torch.cuda.get_device_name(torch.cuda.current_device())
    return f"{name}|prec{prec}|{'hess' if hess else 'grad'}|{size_class(grid, npot)}"


def _load():
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(d):
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def _run(ctx, table, grid, prec, hess, out):
    if hess:
        B.hessian_map(table, grid, 1.0, prec, with_alpha=True, ctx=ctx, out=out)
    else:
        ax, ay = B.grad_map(table, grid, 1.0, prec, ctx=ctx)
        out["ax"].copy_(ax)
        out["ay"].copy_(ay)


def tune_map(ctx: B.Context, table, grid, prec=B.FP64, hess=True, reps=3, use_cache=True,
             cands=None, verbose=False):
    """Pick and install the fastest map launch configuration for this workload.
    Returns (best_tuning, [(tuning, seconds), ...])."""
    npot = int(table["x0"].numel())
    key = _key(prec, hess, grid, npot)
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        best = tuple(cache[key]["tuning"])
        ctx.set_map_tuning(prec, best)
        return best, cache[key].get("results", [])
    nx, ny = int(grid[0]), int(grid[1])
    dt = torch.float64 if prec == B.FP64 else torch.float32
    names = ("hxx", "hxy", "hyy", "ax", "ay")
    ref = {k: torch.empty((ny, nx), dtype=dt, device="cuda") for k in names}
    out = {k: torch.empty_like(v) for k, v in ref.items()}
    ctx.set_map_tuning(prec, DEFAULT)
    _run(ctx, table, grid, prec, hess, ref)
    results = []
    for cand in (cands or candidates()):
        ctx.set_map_tuning(prec, cand)
        _run(ctx, table, grid, prec, hess, out)  # warm-up and check
        torch.cuda.synchronize()
        same = all(torch.equal(out[k], ref[k]) for k in (names if hess else ("ax", "ay")))
        if not same:
            if verbose:
                print("rejected (output differs):", cand)
            continue
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            _run(ctx, table, grid, prec, hess, out)
        ev1.record()
        ev1.synchronize()
        sec = ev0.elapsed_time(ev1) * 1e-3 / reps
        results.append((cand, sec))
        if verbose:
            print(f"{cand}: {sec * 1e3:.3f} ms")
    results.sort(key=lambda r: r[1])
    best = tuple(results[0][0]) if results else DEFAULT
    ctx.set_map_tuning(prec, best)
    if use_cache:
        cache[key] = {"tuning": list(best), "results": [[list(c), s] for c, s in results],
                      "time": time.time()}
        _save(cache)
    return best, results


def tune_chi2(ctx: B.Context, fixed, free, free_off, cat, prec=B.FP64, reps=30, rounds=2,
              choices=(4, 8, 12, 16, 24, 32), verbose=False):
    """Pick and install the number of persistent waves per CU of the batched
    source-plane chi^2 for this batch; every choice must give bit-identical
    chi^2 values.  Each choice is timed over `reps` back-to-back calls after
    three untimed ones (calls of a few tens of microseconds: with a handful
    timed right after an idle GPU the ramp decided the pick), in `rounds`
    passes over the choices, keeping each one's best.  Returns
    (best, [(waves_per_cu, seconds), ...])."""
    ref = None
    best_sec = {}
    for _ in range(rounds):
        for bpc in choices:
            ctx.set_chi2_tuning(bpc)
            out = B.chi2_batch(fixed, free, free_off, cat, prec=prec, ctx=ctx)["chi2"]
            torch.cuda.synchronize()
            if ref is None:
                ref = out.clone()
            elif not torch.equal(out, ref):
                if verbose:
                    print("rejected (output differs):", bpc)
                best_sec[bpc] = None
                continue
            if bpc in best_sec and best_sec[bpc] is None:
                continue
            for _ in range(3):
                B.chi2_batch(fixed, free, free_off, cat, prec=prec, ctx=ctx)
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record()
            for _ in range(reps):
                B.chi2_batch(fixed, free, free_off, cat, prec=prec, ctx=ctx)
            ev1.record()
            ev1.synchronize()
            sec = ev0.elapsed_time(ev1) * 1e-3 / reps
            best_sec[bpc] = min(sec, best_sec.get(bpc) or sec)
            if verbose:
                print(f"waves/CU {bpc}: {sec * 1e6:.1f} us")
    results = [(bpc, sec) for bpc, sec in best_sec.items() if sec is not None]
    results.sort(key=lambda r: r[1])
    best = results[0][0]
    ctx.set_chi2_tuning(best)
    return best, results
