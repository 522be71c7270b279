"""Continuous-batching server for simulation requests.

Requests (model, cube edge, steps, seed) arrive over time.  The scheduler
admits them in arrival order while a batch slot and HBM budget are free
(admission by footprint), keeps every admitted grid resident, and advances
all resident grids together, ``chunk`` steps per tick, through one executor
call; grids that finish leave the batch, their result is read back, and the
freed slots and memory admit newly arrived requests at the next tick.

The host keeps up to ``depth`` ticks in flight (two by default): it launches
tick k+1 (admitting what arrived meanwhile) before it waits for tick
k+1-depth, so the device does not idle while the host does the bookkeeping
between ticks; requests that finished in a tick complete when the host sees
that tick's end.

The scheduler is independent of the executor: ``GpuExecutor`` drives the
library's batched persistent kernel (``rd_batch_*``); ``SimulatedExecutor``
models step durations with a cost model on a virtual clock, so the
scheduling logic can be tested without a GPU.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np


@dataclass
class Completion:
    rid: int
    arrival: float
    admitted: float
    finished: float
    cells: int
    steps: int

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class ServeReport:
    completions: List[Completion]
    makespan: float
    busy: float                      # executor time spent stepping
    ticks: int
    peak_resident: int
    peak_bytes: int
    rejected: int = 0
    results: Dict[int, list] = field(default_factory=dict)

    def latencies(self) -> np.ndarray:
        return np.array([c.latency for c in self.completions])

    def summary(self) -> dict:
        lat = self.latencies()
        work = sum(c.cells * c.steps for c in self.completions)
        return {
            "requests": len(self.completions),
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_latency_s": float(lat.mean()) if len(lat) else None,
            "makespan_s": self.makespan,
            "gcell_updates_per_s": work / self.makespan / 1e9 if self.makespan > 0 else None,
            "busy_fraction": self.busy / self.makespan if self.makespan > 0 else None,
            "ticks": self.ticks,
            "peak_resident": self.peak_resident,
            "peak_bytes": self.peak_bytes,
            "rejected": self.rejected,
        }


class Clock:
    def now(self) -> float:
        return time.perf_counter()

    def sleep_until(self, t: float):
        d = t - self.now()
        if d > 0:
            time.sleep(d)


class VirtualClock(Clock):
    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def sleep_until(self, t: float):
        self.t = max(self.t, t)

    def advance(self, dt: float):
        self.t += dt


def serve(requests: Sequence, arrivals: Sequence[float], executor, max_resident: int,
          hbm_budget: int, chunk: int, clock: Optional[Clock] = None,
          keep_results: bool = False, min_run: int = 1, depth: int = 2,
          admit_per_tick: int = 0) -> ServeReport:
    """Run the continuous-batching loop over ``requests`` arriving at
    ``arrivals`` (seconds after start, non-decreasing).  A tick runs up to
    ``chunk`` steps and stops at the earliest finisher, but runs at least
    ``min_run`` steps: grids that finish inside a tick sit out its remaining
    steps (the batched launch skips them), in exchange for fewer ticks.
    ``admit_per_tick`` (0: no limit) caps the requests admitted between two
    ticks, so that a burst of arrivals is admitted while earlier ticks run
    instead of all before the first one."""
    clock = clock or Clock()
    order = sorted(range(len(requests)), key=lambda i: arrivals[i])
    pending = deque(order)
    t0 = clock.now()
    resident: Dict[int, dict] = {}
    bytes_in_use = 0
    done: List[Completion] = []
    results: Dict[int, list] = {}
    busy = 0.0
    ticks = 0
    peak_res = 0
    peak_bytes = 0
    rejected = 0
    inflight = deque()                  # (tick token, [(rec, output)]) launched, not yet seen done

    def complete(tick):
        nonlocal busy
        token, recs = tick
        busy += executor.wait(token)
        t_fin = clock.now() - t0
        for rec, out in recs:
            req = requests[rec["i"]]
            done.append(Completion(rec["i"], float(arrivals[rec["i"]]), rec["admitted"], t_fin,
                                   executor.cells(req), int(req.steps)))
            if keep_results:
                results[rec["i"]] = out

    while pending or resident or inflight:
        now = clock.now() - t0
        # admission in arrival order, by slot and footprint
        admitted = 0
        while pending and arrivals[pending[0]] <= now and (admit_per_tick <= 0 or admitted < admit_per_tick or not resident):
            i = pending[0]
            need = executor.footprint(requests[i])
            if need > hbm_budget:
                pending.popleft()               # can never fit: reject
                rejected += 1
                continue
            if len(resident) >= max_resident or bytes_in_use + need > hbm_budget:
                break
            pending.popleft()
            h = executor.admit(requests[i])
            resident[h] = {"i": i, "admitted": clock.now() - t0, "bytes": need,
                           "left": int(requests[i].steps)}
            bytes_in_use += need
            admitted += 1
        peak_res = max(peak_res, len(resident))
        peak_bytes = max(peak_bytes, bytes_in_use)
        launched = None
        if resident:
            # one tick: advance every resident grid by up to `run` steps; `run`
            # stops at the earliest finisher so no grid idles in the batch
            run = min(chunk, max(min_run, min(r["left"] for r in resident.values())))
            finished = executor.step(run)
            token = executor.mark()
            recs = []
            for h in finished:
                rec = resident.pop(h)
                recs.append((rec, executor.collect(h, keep_results)))
                bytes_in_use -= rec["bytes"]
            for r in resident.values():
                r["left"] -= run
                assert r["left"] > 0, "the executor did not report a finished grid"
            ticks += 1
            launched = (token, recs)
        if launched:
            inflight.append(launched)
        while inflight and (len(inflight) > max(1, depth) or not resident):
            complete(inflight.popleft())
        if not resident and not inflight and pending:
            clock.sleep_until(t0 + arrivals[pending[0]])
    makespan = clock.now() - t0
    return ServeReport(done, makespan, busy, ticks, peak_res, peak_bytes, rejected, results)


class SimulatedExecutor:
    """Cost-model executor on a virtual clock: a tick of `run` steps over the
    resident grids takes launch_s + run * (cells_resident / rate) seconds of
    device time; ticks queue on the device in launch order, and waiting for
    one advances the clock to its end."""

    def __init__(self, clock: VirtualClock, rate_cells_per_s: float = 3e11, launch_s: float = 2e-5,
                 bytes_per_cell: int = 8):
        self.clock = clock
        self.rate = rate_cells_per_s
        self.launch = launch_s
        self.bpc = bytes_per_cell
        self.live: Dict[int, dict] = {}
        self.next = 0
        self.free_at = 0.0              # when the device finishes its queued ticks

    def cells(self, req) -> int:
        return req.edge ** 3

    def footprint(self, req) -> int:
        ns = 2 if req.model == "brusselator" else 1
        return 2 * ns * self.cells(req) * 4

    def admit(self, req) -> int:
        h = self.next
        self.next += 1
        self.live[h] = {"req": req, "left": int(req.steps)}
        return h

    def step(self, run: int) -> List[int]:
        cells = sum(self.cells(v["req"]) for v in self.live.values())
        cost = self.launch + run * cells / self.rate
        self.free_at = max(self.free_at, self.clock.now()) + cost
        self.last = (self.free_at, cost)
        fin = []
        for h, v in list(self.live.items()):
            v["left"] -= min(run, v["left"])
            if v["left"] == 0:
                fin.append(h)
        return fin

    def collect(self, h: int, keep: bool):
        self.live.pop(h)
        return None

    def mark(self):
        """Token of the tick just launched: (end time, device time)."""
        return self.last

    def wait(self, token) -> float:
        end, cost = token
        self.clock.sleep_until(end)
        return cost


class GpuExecutor:
    """Drives rd_batch_*: one persistent batched launch per step, a captured
    hipGraph per tick length; grids are pooled by (edge, model) and reused."""

    def __init__(self, storage: str = "f32", max_resident: int = 512, hbm_budget: int = 1 << 36,
                 stream=None):
        import torch

        from . import rd
        from . import workloads as W
        self.rd, self.W, self.torch = rd, W, torch
        self.storage = storage
        self.stream = stream or torch.cuda.Stream()
        self.batch = rd.Batch(max_resident, hbm_budget, storage, stream=self.stream)
        self.pool: Dict[tuple, list] = {}
        self.by_handle: Dict[int, tuple] = {}
        self.grid_of: Dict[int, object] = {}

    def cells(self, req) -> int:
        return req.edge ** 3

    def footprint(self, req) -> int:
        ns = 2 if req.model == "brusselator" else 1
        return self.rd.grid_bytes((req.edge,) * 3, ns, self.storage)

    def admit(self, req) -> int:
        key = (req.edge, req.model)
        free = self.pool.setdefault(key, [])
        if free:
            g = free.pop()
        else:
            g = self.rd.Grid((req.edge,) * 3, 2 if req.model == "brusselator" else 1, 1.0,
                             self.storage, stream=self.stream)
            g.set_model(self.W.request_spec(req))
        with self.torch.cuda.stream(self.stream):      # same stream as the grid's copies
            fields = self.W.request_fields_device(req)
            # enqueued behind the ticks in flight: the tensors are freed to
            # torch's pool for this stream, which reuses them in stream order
            for s, f in enumerate(fields):
                g.write(s, f, enqueue_only=True)
        self.batch.add(g, int(req.steps))
        h = g.handle.value
        self.by_handle[h] = key
        self.grid_of[h] = g
        return h

    def step(self, run: int) -> List[int]:
        self._start = self.torch.cuda.Event(enable_timing=True)
        self._start.record(self.stream)
        return [g.handle.value for g in self.batch.step(run)]

    def mark(self):
        """Events around the tick just launched on the executor's stream."""
        end = self.torch.cuda.Event(enable_timing=True)
        end.record(self.stream)
        return (self._start, end)

    def wait(self, token) -> float:
        """Block until the tick has run; its device time in seconds."""
        start, end = token
        end.synchronize()
        return start.elapsed_time(end) * 1e-3

    def collect(self, h: int, keep: bool):
        # a pooled grid is reused on the same stream, after this tick's launch
        g = self.grid_of.pop(h)
        out = g.read_all(np.float32) if keep else None
        self.pool[self.by_handle.pop(h)].append(g)
        return out

    def close(self):
        self.batch.close()
        for lst in self.pool.values():
            for g in lst:
                g.close()
        self.pool.clear()


def poisson_arrivals(trace, rate_per_s: float) -> np.ndarray:
    """Arrival times (s) from the trace's unit-rate exponential gaps."""
    gaps = np.array([r.gap for r in trace]) / rate_per_s
    return np.cumsum(gaps) - gaps[0]
