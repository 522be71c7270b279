"""Scheduler tests on a simulated executor (virtual clock, cost model): no GPU."""
import numpy as np

from paper_1004_0480_amd import serve as S
from paper_1004_0480_amd import workloads as W


def run(trace, arrivals, max_resident=64, budget=1 << 40, chunk=50, rate=3e11):
    clock = S.VirtualClock()
    ex = S.SimulatedExecutor(clock, rate_cells_per_s=rate)
    rep = S.serve(trace, arrivals, ex, max_resident, budget, chunk, clock=clock)
    return rep, ex


def small_trace(n=60, seed=7):
    return W.make_trace(n, seed=seed, edges=(32, 48, 64), min_steps=50, max_steps=400)


def test_every_request_completes_once_with_sane_times():
    tr = small_trace()
    arr = S.poisson_arrivals(tr, 2000.0)
    rep, _ = run(tr, arr)
    ids = sorted(c.rid for c in rep.completions)
    assert ids == list(range(len(tr)))
    for c in rep.completions:
        assert c.arrival <= c.admitted <= c.finished
        assert c.latency > 0
    s = rep.summary()
    assert s["p50_latency_s"] <= s["p99_latency_s"]
    assert 0 < s["busy_fraction"] <= 1.0 + 1e-9


def test_slot_and_budget_limits_hold():
    tr = small_trace()
    arr = np.zeros(len(tr))
    ex_bytes = S.SimulatedExecutor(S.VirtualClock()).footprint
    budget = 3 * max(ex_bytes(r) for r in tr)
    rep, _ = run(tr, arr, max_resident=5, budget=budget)
    assert rep.peak_resident <= 5
    assert rep.peak_bytes <= budget
    assert len(rep.completions) == len(tr)


def test_oversized_request_is_rejected_not_stuck():
    tr = small_trace(10)
    big = W.Request(99, 0.1, 128, "brusselator", 100, 1)
    tr = tr + [big]
    arr = np.linspace(0, 0.001, len(tr))
    ex_bytes = S.SimulatedExecutor(S.VirtualClock()).footprint
    budget = max(ex_bytes(r) for r in tr[:-1]) * 2
    rep, _ = run(tr, arr, budget=budget)
    assert rep.rejected == 1
    assert len(rep.completions) == len(tr) - 1


def test_continuous_batching_admits_while_others_run():
    """A request arriving while an earlier one is on the device is admitted
    before the earlier one finishes (work overlaps), unlike a one-at-a-time queue."""
    tr = [W.Request(0, 0, 64, "diffusion", 2000, 1), W.Request(1, 0, 32, "diffusion", 100, 2)]
    arr = np.array([0.0, 1e-4])
    rep, _ = run(tr, arr, chunk=10)
    c = {x.rid: x for x in rep.completions}
    assert c[1].admitted < c[0].finished
    assert c[1].finished < c[0].finished        # the short late request overtakes


def test_batching_beats_serial_queue_on_latency():
    tr = small_trace(80)
    arr = S.poisson_arrivals(tr, 3000.0)
    batched, _ = run(tr, arr, max_resident=64)
    serial, _ = run(tr, arr, max_resident=1)
    assert batched.summary()["p99_latency_s"] < serial.summary()["p99_latency_s"]
    assert batched.summary()["mean_latency_s"] < serial.summary()["mean_latency_s"]


def test_ticks_stop_at_the_earliest_finisher():
    tr = [W.Request(0, 0, 32, "diffusion", 30, 1), W.Request(1, 0, 32, "diffusion", 75, 2)]
    rep, _ = run(tr, np.zeros(2), chunk=50)
    # ticks of 30, then 45 steps
    assert rep.ticks == 2


def test_minimum_tick_length_merges_close_finishers():
    """With min_run, grids that finish within a few steps of each other leave
    in one tick (they sit out its remaining steps); every request still
    completes exactly once."""
    tr = [W.Request(i, 0, 32, "diffusion", st, i) for i, st in enumerate([20, 22, 24, 26, 100])]
    clock = S.VirtualClock()
    ex = S.SimulatedExecutor(clock)
    rep = S.serve(tr, np.zeros(len(tr)), ex, 64, 1 << 40, 50, clock=clock, min_run=8)
    assert rep.ticks == 4                       # 20, 8 (three finish), 50, 22
    assert sorted(c.rid for c in rep.completions) == list(range(len(tr)))
    rep1, _ = run(tr, np.zeros(len(tr)))
    assert rep1.ticks == 6                      # 20, 2, 2, 2, 50, 22


def test_deeper_pipelining_keeps_every_request_and_ordering():
    """One, two or three ticks in flight: every request completes once, after
    it arrived and was admitted, and the device time never exceeds the
    makespan."""
    tr = small_trace(50)
    arr = S.poisson_arrivals(tr, 2500.0)
    for depth in (1, 2, 3):
        clock = S.VirtualClock()
        ex = S.SimulatedExecutor(clock)
        rep = S.serve(tr, arr, ex, 16, 1 << 40, 50, clock=clock, depth=depth)
        assert sorted(c.rid for c in rep.completions) == list(range(len(tr)))
        for c in rep.completions:
            assert c.arrival <= c.admitted <= c.finished
        assert 0 < rep.summary()["busy_fraction"] <= 1.0 + 1e-9


def test_admission_cap_spreads_a_burst_over_ticks():
    """All requests at t = 0 with at most 4 admitted between ticks: the
    batch fills over several ticks, every request still completes once, and
    the cap never stops admission into an empty batch."""
    class Recording(S.SimulatedExecutor):
        def step(self, run):
            self.sizes.append(len(self.live))
            return super().step(run)

    tr = small_trace(30)
    clock = S.VirtualClock()
    ex = Recording(clock)
    ex.sizes = []
    rep = S.serve(tr, np.zeros(len(tr)), ex, 16, 1 << 40, 50, clock=clock, admit_per_tick=4)
    assert sorted(c.rid for c in rep.completions) == list(range(len(tr)))
    assert ex.sizes[:3] == [4, 8, 12]                      # the batch fills four at a time
    assert max(ex.sizes) <= 16
    assert rep.peak_resident <= 16


def test_trace_statistics():
    tr = W.make_trace(4096, seed=4)
    edges = np.array([r.edge for r in tr])
    steps = np.array([r.steps for r in tr])
    brus = np.mean([r.model == "brusselator" for r in tr])
    assert set(edges) == set(W.SERVE_EDGES)
    assert steps.min() >= 200 and steps.max() <= 2000
    assert abs(brus - 0.5) < 0.03
    assert abs(np.mean([r.gap for r in tr]) - 1.0) < 0.05
    assert len({r.seed for r in tr}) == len(tr)
