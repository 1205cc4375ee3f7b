"""The serving scheduler on a scripted device (no GPU): admission by slots and
HBM footprint, deferral, chi^2 merging, overlap of requests, latency stats."""
import pytest

from paper_2004_06352_amd.serve import FakeBackend, Req, Scheduler, ScriptedClock


def make(clock, budget=1000, dur=None, fp=None):
    dur = dur or (lambda g: 0.010 if g[0].kind == "map" else 0.001 * len(g))
    fp = fp or (lambda g: 100 if g[0].kind == "map" else 10 * len(g))
    return FakeBackend(clock, dur, fp, budget)


def overlaps(launched, dur_of):
    """Largest number of launches running at one instant."""
    ev = []
    for t, slot, ids in launched:
        ev.append((t, 1))
        ev.append((t + dur_of(ids), -1))
    ev.sort(key=lambda e: (e[0], e[1]))
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


def test_all_requests_complete_with_consistent_times():
    clock = ScriptedClock()
    be = make(clock)
    reqs = [Req(i, 0.002 * i, "map", side=512, model=0, npot=10) for i in range(20)]
    st = Scheduler(be, n_slots=2).run(reqs, clock=clock, sleep=clock.sleep)
    assert st["requests"] == 20
    for r in reqs:
        assert r.admitted >= r.t and r.done >= r.admitted + 0.010 - 1e-9
    assert st["p99_ms"] >= st["p50_ms"] >= 10.0 - 1e-6


def test_slots_bound_concurrency_and_work_overlaps():
    clock = ScriptedClock()
    be = make(clock)
    reqs = [Req(i, 0.0, "map", side=512, model=0, npot=10) for i in range(9)]
    Scheduler(be, n_slots=3).run(reqs, clock=clock, sleep=clock.sleep)
    assert overlaps(be.launched, lambda ids: 0.010) == 3


def test_continuous_admission_of_late_arrivals():
    """A request arriving while another is on the device starts before the
    first one finishes when a slot is free."""
    clock = ScriptedClock()
    be = make(clock)
    a = Req(0, 0.0, "map", side=512, model=0, npot=10)
    b = Req(1, 0.004, "map", side=512, model=0, npot=10)
    Scheduler(be, n_slots=2).run([a, b], clock=clock, sleep=clock.sleep)
    assert b.admitted < a.done


def test_memory_budget_defers_and_is_never_exceeded():
    clock = ScriptedClock()
    be = make(clock, budget=250)  # two maps fit, the third waits
    reqs = [Req(i, 0.0, "map", side=512, model=0, npot=10) for i in range(6)]
    st = Scheduler(be, n_slots=4).run(reqs, clock=clock, sleep=clock.sleep)
    assert st["deferred"] >= 1
    assert st["peak_bytes"] <= 250
    assert overlaps(be.launched, lambda ids: 0.010) == 2


def test_request_larger_than_budget_is_refused():
    clock = ScriptedClock()
    be = make(clock, budget=50)
    with pytest.raises(MemoryError):
        Scheduler(be).run([Req(0, 0.0, "map", side=512)], clock=clock, sleep=clock.sleep)


def test_waiting_chi2_requests_are_merged_up_to_the_sample_limit():
    clock = ScriptedClock()
    be = make(clock)
    first = Req(0, 0.0, "map", side=512, model=0, npot=10)
    chis = [Req(i, 0.001, "chi2", samples=100) for i in range(1, 8)]
    Scheduler(be, n_slots=1, max_merge_samples=300).run([first] + chis, clock=clock,
                                                        sleep=clock.sleep)
    groups = [ids for _, _, ids in be.launched]
    assert groups[0] == [0]
    assert groups[1:] == [[1, 2, 3], [4, 5, 6], [7]]


def test_no_merging_when_disabled():
    clock = ScriptedClock()
    be = make(clock)
    chis = [Req(i, 0.0, "chi2", samples=100) for i in range(4)]
    Scheduler(be, n_slots=1, merge_chi2=False).run(chis, clock=clock, sleep=clock.sleep)
    assert [ids for _, _, ids in be.launched] == [[0], [1], [2], [3]]


def test_results_are_kept_when_asked():
    clock = ScriptedClock()
    be = make(clock)
    reqs = [Req(i, 0.0, "chi2", samples=5) for i in range(3)]
    Scheduler(be, n_slots=2, keep_results=True).run(reqs, clock=clock, sleep=clock.sleep)
    assert [r.result for r in reqs] == [("done", 0), ("done", 1), ("done", 2)]


def test_request_stream_generator():
    from paper_2004_06352_amd import inputs
    rs = inputs.config5_requests(n_requests=200, rate_hz=50.0)
    kinds = {r["kind"] for r in rs}
    assert kinds == {"map", "chi2"}
    ts = [r["t"] for r in rs]
    assert ts == sorted(ts)
    assert all(64 <= r["samples"] <= 4096 for r in rs if r["kind"] == "chi2")
    assert all(r["side"] in (512, 1024, 2048, 4096) for r in rs if r["kind"] == "map")
    assert all(50 <= r["npot"] <= 1000 for r in rs if r["kind"] == "map")
    Req.from_dict(rs[0])


def test_merging_stops_at_the_memory_budget():
    """Six waiting chi^2 requests of 10 B each under a 50 B budget: the merged
    batch takes the five that fit and the sixth runs after it; no request is
    refused, the budget is never exceeded."""
    clock = ScriptedClock()
    be = make(clock, budget=50)
    chis = [Req(i, 0.0, "chi2", samples=10) for i in range(6)]
    st = Scheduler(be, n_slots=2).run(chis, clock=clock, sleep=clock.sleep)
    assert [ids for _, _, ids in be.launched] == [[0, 1, 2, 3, 4], [5]]
    assert st["peak_bytes"] <= 50 and all(r.done is not None for r in chis)


def test_head_chi2_request_over_the_free_room_waits():
    """A map holds most of the budget; the chi^2 request behind it is not
    merged beyond the room left and waits for the map to finish."""
    clock = ScriptedClock()
    be = make(clock, budget=120)
    reqs = [Req(0, 0.0, "map", side=512, model=0, npot=10)] + \
        [Req(i, 0.0, "chi2", samples=10) for i in range(1, 4)]
    st = Scheduler(be, n_slots=2).run(reqs, clock=clock, sleep=clock.sleep)
    groups = [ids for _, _, ids in be.launched]
    assert groups[0] == [0] and groups[1] == [1, 2]
    assert st["peak_bytes"] <= 120


def test_scratch_accounting_with_the_library_sizes():
    """The slots' context scratch is sized by the library (host arithmetic,
    no device) for the largest map and merged chi^2 batch, reserved up front,
    and the requests' own buffers are charged against what remains: with a
    device share that holds the reservation plus two maps, a third map
    waits, and reservation + peak never exceed the share."""
    from paper_2004_06352_amd import binding as B
    from paper_2004_06352_amd import inputs
    from paper_2004_06352_amd.serve import HbmAccount
    c3 = inputs.config3(n_samples=1)
    nsys, nimg = len(c3["catalog"]["off"]) - 1, int(c3["catalog"]["off"][-1])
    acc = HbmAccount(B.map_scratch_bytes, B.chi2_scratch_bytes, 4, 300, nsys, nimg,
                     inputs.N_FREE, 16384, 1000)
    # the library's layout: derived constants of 35 doubles + 19 floats per
    # potential (tables padded to 64 entries), per-image constants
    assert B.map_scratch_bytes(1000) == 1024 * 356
    chi2 = B.chi2_scratch_bytes(300, 16384 * 6, 16384, nsys, nimg)
    assert chi2 >= 320 * 356 + 16384 * 6 * 356 + 3 * nimg * 8
    assert acc.slot_scratch == max(1024 * 356, chi2) and acc.reserved == 4 * acc.slot_scratch
    with pytest.raises(MemoryError):
        acc.budget(acc.reserved)
    map_b = HbmAccount.map_bytes(1024, 8)
    share = acc.reserved + 2 * map_b + map_b // 2
    clock = ScriptedClock()
    be = FakeBackend(clock, lambda g: 0.01,
                     lambda g: (HbmAccount.map_bytes(g[0].side, 8) if g[0].kind == "map"
                                else HbmAccount.chi2_bytes(sum(r.samples for r in g),
                                                           6 * sum(r.samples for r in g))),
                     acc.budget(share))
    reqs = [Req(i, 0.0, "map", side=1024, model=0, npot=100) for i in range(3)] + \
        [Req(3, 0.0, "chi2", samples=4096)]
    st = Scheduler(be, n_slots=4).run(reqs, clock=clock, sleep=clock.sleep)
    assert st["deferred"] >= 1 and acc.reserved + st["peak_bytes"] <= share
