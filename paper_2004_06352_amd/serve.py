"""Serving loop for lens maps and chi^2 batches with continuous batching.

Requests (maps of a resident lens model at some grid size; chi^2 batches of
model samples) arrive over time.  The scheduler

  * keeps the lens models, the chi^2 fixed model and the constraint catalogue
    resident on the device,
  * admits the oldest waiting request as soon as a launch slot is free and its
    HBM footprint fits the budget (head-of-line order; a request that cannot
    fit is counted as deferred and waits for completions to free memory),
  * merges waiting chi^2 requests into one batched launch when a chi^2 request
    reaches the head of the queue, up to a sample limit and to what the memory
    budget still holds,
  * charges each slot's library scratch to the budget up front, sized by the
    library's own layout (`HbmAccount`), and each request's buffers while it
    is in flight,
  * runs admitted work on several streams at once, so requests that arrive
    while others are on the GPU overlap with them on the device,
  * records arrival, admission and completion times, from which it reports
    p50/p99 latency and throughput.

The scheduling logic is independent of the device: `Scheduler` drives any
backend with footprint/launch/poll/finish, so it is tested on the CPU with a
scripted clock (`FakeBackend`) and runs the library through `GpuBackend`.
Every request's result is computed by the same kernels whether it runs alone
or in a mix, so it is the same bit for bit.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass
from typing import Any, Callable, List, Optional

import numpy as np


@dataclass
class Req:
    id: int
    t: float                 # arrival time [s] from the start of the stream
    kind: str                # "map" or "chi2"
    side: int = 0
    model: int = -1
    npot: int = 0
    model_seed: int = 0
    samples: int = 0
    seed: int = 0
    admitted: Optional[float] = None
    done: Optional[float] = None
    result: Any = None

    @staticmethod
    def from_dict(d):
        return Req(**{k: v for k, v in d.items() if k in Req.__dataclass_fields__})


class Scheduler:
    def __init__(self, backend, n_slots=4, hbm_budget=None, merge_chi2=True,
                 max_merge_samples=16384, keep_results=False):
        self.backend = backend
        self.n_slots = n_slots
        self.budget = hbm_budget if hbm_budget is not None else backend.default_budget()
        self.merge_chi2 = merge_chi2
        self.max_merge_samples = max_merge_samples
        self.keep_results = keep_results

    def _group(self, queue, room):
        """The head request, and when it is a chi^2 batch every later waiting
        chi^2 request that keeps the merged batch within the sample limit and
        its footprint within `room` (the budget not in use)."""
        head = queue[0]
        if head.kind != "chi2" or not self.merge_chi2:
            return [head]
        group, n = [head], head.samples
        for r in list(queue)[1:]:
            if r.kind != "chi2":
                continue
            if n + r.samples > self.max_merge_samples:
                break
            if self.backend.footprint(group + [r]) > room:
                break
            group.append(r)
            n += r.samples
        return group

    def run(self, reqs: List[Req], clock: Callable[[], float] = time.perf_counter,
            sleep: Callable[[float], None] = time.sleep, idle: float = 2e-5):
        pending = collections.deque(sorted(reqs, key=lambda r: (r.t, r.id)))
        queue = collections.deque()
        inflight = {}
        free_slots = list(range(self.n_slots))
        used = peak = 0
        deferred_ids = set()
        launches = merged = 0
        max_inflight = 0
        t0 = clock()
        while pending or queue or inflight:
            now = clock() - t0
            progressed = False
            while pending and pending[0].t <= now:
                queue.append(pending.popleft())
                progressed = True
            for slot in list(inflight):
                ticket, group, nbytes = inflight[slot]
                if self.backend.poll(ticket):
                    results = self.backend.finish(ticket)
                    t_done = clock() - t0
                    for r, res in zip(group, results):
                        r.done = t_done
                        r.result = res if self.keep_results else None
                    used -= nbytes
                    del inflight[slot]
                    free_slots.append(slot)
                    progressed = True
            while queue and free_slots:
                group = self._group(queue, self.budget - used)
                need = self.backend.footprint(group)
                if need > self.budget:  # the head alone: it can never run
                    raise MemoryError(f"request {group[0].id} needs {need} B > budget {self.budget} B")
                if used + need > self.budget:
                    deferred_ids.add(group[0].id)
                    break
                ids = {r.id for r in group}
                queue = collections.deque(r for r in queue if r.id not in ids)
                slot = free_slots.pop(0)
                t_adm = clock() - t0
                for r in group:
                    r.admitted = t_adm
                inflight[slot] = (self.backend.launch(group, slot), group, need)
                used += need
                peak = max(peak, used)
                launches += 1
                merged += len(group) - 1
                max_inflight = max(max_inflight, len(inflight))
                progressed = True
            if not progressed:
                sleep(idle)
        return self.stats(reqs, deferred=len(deferred_ids), launches=launches, merged=merged,
                          peak_bytes=peak, max_inflight=max_inflight)

    def stats(self, reqs, **extra):
        lat = np.array([r.done - r.t for r in reqs])
        span = max(r.done for r in reqs) - min(r.t for r in reqs) if reqs else 0.0
        out = dict(requests=len(reqs), p50_ms=float(np.percentile(lat, 50) * 1e3) if len(lat) else 0,
                   p99_ms=float(np.percentile(lat, 99) * 1e3) if len(lat) else 0,
                   mean_ms=float(lat.mean() * 1e3) if len(lat) else 0,
                   span_s=float(span), req_per_s=len(reqs) / span if span > 0 else 0.0)
        for kind in ("map", "chi2"):
            sel = [r for r in reqs if r.kind == kind]
            if sel:
                l = np.array([r.done - r.t for r in sel])
                out[f"{kind}_p50_ms"] = float(np.percentile(l, 50) * 1e3)
                out[f"{kind}_p99_ms"] = float(np.percentile(l, 99) * 1e3)
        evals = sum(r.side * r.side * r.npot for r in reqs if r.kind == "map")
        samples = sum(r.samples for r in reqs if r.kind == "chi2")
        out["map_evals_per_s"] = evals / span if span > 0 else 0.0
        out["chi2_samples_per_s"] = samples / span if span > 0 else 0.0
        out.update(extra)
        return out


# ---------------------------------------------------------------------------
class FakeBackend:
    """Scripted device for testing the scheduler without a GPU: each launch
    takes `duration(group)` seconds of the scheduler's clock and occupies
    `footprint(group)` bytes."""

    def __init__(self, clock, duration, footprint, budget=1 << 30):
        self.clock = clock
        self.duration = duration
        self._footprint = footprint
        self._budget = budget
        self.launched = []

    def default_budget(self):
        return self._budget

    def footprint(self, group):
        return self._footprint(group)

    def launch(self, group, slot):
        end = self.clock() + self.duration(group)
        self.launched.append((self.clock(), slot, [r.id for r in group]))
        return (end, group)

    def poll(self, ticket):
        return self.clock() >= ticket[0]

    def finish(self, ticket):
        return [("done", r.id) for r in ticket[1]]


class ScriptedClock:
    """A clock that only advances when the scheduler sleeps."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


# ---------------------------------------------------------------------------
class HbmAccount:
    """The device memory the serving loop charges against its budget.

    Each slot's library context holds scratch that persists between requests
    (derived tables, per-image constants): it is reserved up front, sized by
    the library's own layout (lens_map_scratch_bytes, lens_chi2_scratch_bytes)
    for the largest request a slot may run -- a map of `max_map_pots`
    potentials or a merged chi^2 batch of `max_merge_samples` samples -- and
    the context is created with that limit.  A request in flight is charged
    its own buffers: a map its five output planes; a chi^2 batch its free
    potentials (physical and amplitude tables, 7 doubles each), offsets and
    chi^2 values."""

    def __init__(self, map_scratch, chi2_scratch, n_slots, n_fixed, n_sys, n_img,
                 free_per_sample, max_merge_samples, max_map_pots):
        self.slot_scratch = max(
            map_scratch(max_map_pots),
            chi2_scratch(n_fixed, max_merge_samples * free_per_sample, max_merge_samples, n_sys,
                         n_img))
        self.reserved = n_slots * self.slot_scratch

    def budget(self, device_bytes):
        """Budget left for requests out of `device_bytes` for the server."""
        b = int(device_bytes) - self.reserved
        if b <= 0:
            raise MemoryError(f"{device_bytes} B cannot hold the slots' scratch ({self.reserved} B)")
        return b

    @staticmethod
    def map_bytes(side, elem_size):
        return 5 * side * side * elem_size

    @staticmethod
    def chi2_bytes(n_samples, n_free):
        return n_free * 2 * 7 * 8 + (n_samples + 1) * 4 + n_samples * 8


class GpuBackend:
    """Runs requests through the C library.  One (stream, context) pair per
    slot; lens models, the chi^2 fixed model and the catalogue are uploaded
    once and stay resident."""

    def __init__(self, n_slots=4, prec=0, models=None, map_range=(-100.0, 100.0),
                 chi2_model=None, zs_map=2.0, max_merge_samples=16384, max_map_pots=1000):
        import torch

        from . import binding as B
        from . import inputs
        self.torch, self.B, self.inputs = torch, B, inputs
        self.prec = prec
        c3 = chi2_model or inputs.config3(n_samples=1)
        cat = c3["catalog"]
        self.account = HbmAccount(B.map_scratch_bytes, B.chi2_scratch_bytes, n_slots,
                                  len(c3["fixed"]["x0"]), len(cat["off"]) - 1,
                                  int(cat["off"][-1]), inputs.N_FREE, max_merge_samples,
                                  max_map_pots)
        dev = torch.cuda.current_device()
        self.slots = [(torch.cuda.Stream(),
                       B.Context(dev, scratch_max=self.account.slot_scratch, check=False))
                      for _ in range(n_slots)]
        self.map_range = map_range
        self.f_map = B.dlsds(inputs.ZL, zs_map)
        self.models = {}
        for mid, (npot, seed) in enumerate(models or []):
            phys = B.to_device(inputs.map_request_pots(npot, seed), B.PHYS_KEYS)
            self.models[mid] = B.table_from_physical(phys, 0, self.slots[0][1])
        self.fixed = B.table_from_physical(B.to_device(c3["fixed"], B.PHYS_KEYS), 0,
                                           self.slots[0][1])
        self.cat = B.catalog_to_device(B.catalog_with_dlsds(c3["catalog"], c3["zl"]))
        self._payload = {}
        torch.cuda.synchronize()

    def default_budget(self):
        free, total = self.torch.cuda.mem_get_info()
        return self.account.budget(0.5 * free)

    # host payload of a chi^2 request: its samples drawn from the priors
    # (what a client sends); prepare() builds them before the stream starts
    def chi2_samples(self, r):
        if r.id in self._payload:
            return self._payload[r.id]
        rng = np.random.default_rng(r.seed)
        return self.inputs.draw_samples(rng, r.samples)

    def prepare(self, reqs):
        self._payload = {r.id: self.chi2_samples(r) for r in reqs if r.kind == "chi2"}

    def footprint(self, group):
        if group[0].kind == "map":
            return HbmAccount.map_bytes(group[0].side, 8 if self.prec == 0 else 4)
        n = sum(r.samples for r in group)
        nfree = sum(len(self.chi2_samples(r)[0]["x0"]) for r in group)
        return HbmAccount.chi2_bytes(n, nfree)

    def grid(self, side):
        lo, hi = self.map_range
        d = (hi - lo) / side
        return (side, side, lo + 0.5 * d, lo + 0.5 * d, d, d)

    def launch(self, group, slot):
        torch, B = self.torch, self.B
        stream, ctx = self.slots[slot]
        with torch.cuda.stream(stream):
            if group[0].kind == "map":
                r = group[0]
                out = B.hessian_map(self.models[r.model], self.grid(r.side), self.f_map, self.prec,
                                    with_alpha=True, ctx=ctx)
                results = [out]
            else:
                frees, offs = [], [0]
                for r in group:
                    free, off = self.chi2_samples(r)
                    frees.append(free)
                    offs.extend((off[1:] + offs[-1]).tolist())
                free = {k: np.concatenate([f[k] for f in frees]) for k in self.inputs.PHYS_KEYS}
                pinned = {k: torch.from_numpy(v).pin_memory() for k, v in free.items()}
                phys = {k: v.to("cuda", non_blocking=True) for k, v in pinned.items()}
                off_t = torch.tensor(offs, dtype=torch.int32).pin_memory().to("cuda",
                                                                               non_blocking=True)
                table = B.table_from_physical(phys, 0, ctx)
                res = B.chi2_batch(self.fixed, table, off_t, self.cat, prec=self.prec, ctx=ctx)
                chi2 = res["chi2"]
                results, at = [], 0
                for r in group:
                    results.append(chi2[at:at + r.samples])
                    at += r.samples
                inputs_alive = (pinned, phys, off_t, table)
            ev = torch.cuda.Event()
            ev.record(stream)
        if group[0].kind == "map":
            inputs_alive = None
        # the ticket holds the request's inputs until it completes
        return (ev, results, stream, inputs_alive)

    def poll(self, ticket):
        return ticket[0].query()

    def finish(self, ticket):
        return ticket[1]
