"""GPU parity after the configured step counts, element by element.

Each test runs the HIP path in the plan the benchmark uses (autotuned) and
the FP64 oracle on the same seeded input, then checks every species:
  - relative L2 error <= 1e-5 (the FP32 target, section 2's Eq. (5) stepped
    the configured number of times);
  - the largest element error <= 10 x 1e-5 x max|oracle|.  An FP32 step
    rounds each cell's update a few times, and these errors add up smoothly
    over the grid, so the worst cell stays within a small factor of the RMS
    error; a defect confined to a tile edge, a face or a plane (a wrong
    neighbour, a dropped term) makes errors of order dt |R| there, far above
    this bound, while it could hide below the L2 norm of a large grid.
BF16 storage is reported against the same FP64 oracle (both rounding modes)
and held to bounds twice the measured errors.
"""
import numpy as np
import pytest

import oracle
from paper_1004_0480_amd import rd
from paper_1004_0480_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5
MAX_FACTOR = 10.0
# front384 BF16 storage after 100 steps against FP64, per species (A, B, C):
# (rel-L2, max-abs) bounds, twice the errors measured on MI355X
BF16_NEAREST = [(2.0e-2, 2.1e-2), (1.5e-2, 1.9e-2), (3.5e-3, 7.6e-2)]
BF16_STOCHASTIC = [(4.9e-3, 2.5e-2), (4.9e-3, 9.3e-3), (7.2e-4, 5.8e-2)]


def errors(got, ref):
    d = got - ref
    return float(np.linalg.norm(d) / np.linalg.norm(ref)), float(np.max(np.abs(d))), float(np.max(np.abs(ref)))


def run_autotuned(w, steps, storage="f32", rounding=None, plan=None):
    g = rd.Grid.from_workload(w, storage=storage)
    if rounding:
        g.set_rounding(rounding, 1)
    if plan:
        g.set_plan(**plan)
    else:
        g.autotune(2)
    g.step(steps)
    out = g.read_all()
    used = g.plan()
    g.close()
    return out, used


def check_fp32(name, w, steps, got, ref, plan, tol=None):
    """tol: per-species rel-L2 bounds where FP32 itself cannot reach TOL."""
    for s in range(w.spec.ns):
        e, m, scale = errors(got[s], ref[s])
        t = tol[s] if tol else TOL
        print("%s %s %d steps species %d: rel-L2 %.3e max-abs %.3e (max |ref| %.3e) plan %s"
              % (name, w.shape, steps, s, e, m, scale, plan), flush=True)
        assert e <= t, (name, s, e)
        assert m <= MAX_FACTOR * TOL * scale, (name, s, m)


@pytest.mark.timeout(900)
def test_brusselator256_full_run():
    """The 256^3 Brusselator for its configured 2000 steps."""
    w = W.make_workload("brusselator256")
    got, plan = run_autotuned(w, w.steps)
    ref = oracle.run(w.spec, w.fields, w.steps)
    check_fp32("brusselator256", w, w.steps, got, ref, plan)


@pytest.mark.timeout(900)
def test_front384_full_size_fp32_and_bf16():
    """front384 at full size, 100 steps (the oracle's share of a test run):
    FP32 in the one-pass plan to the FP32 bounds; BF16 storage with
    round-to-nearest and with stochastic rounding reported per field."""
    w = W.make_workload("front384")
    steps = 100
    ref = oracle.run(w.spec, w.fields, steps)
    got, plan = run_autotuned(w, steps)
    assert plan["kernel"] == rd.KERNEL["fused"], plan
    check_fp32("front384", w, steps, got, ref, plan)
    del got
    # (rel-L2, max-abs) per species: twice the errors measured on MI355X
    bounds = {"nearest": BF16_NEAREST, "stochastic": BF16_STOCHASTIC}
    found = {}
    for mode in ("nearest", "stochastic"):
        got, plan = run_autotuned(w, steps, storage="bf16", rounding=mode)
        for s in range(3):
            e, m, scale = errors(got[s], ref[s])
            found[mode, s] = (e, m)
            print("front384 BF16 %s %d steps species %d: rel-L2 %.3e max-abs %.3e plan %s"
                  % (mode, steps, s, e, m, plan), flush=True)
        del got
    for (mode, s), (e, m) in found.items():
        assert e <= bounds[mode][s][0] and m <= bounds[mode][s][1], (mode, s, e, m)


@pytest.mark.timeout(900)
def test_front_configured_steps_reduced_grid():
    """The front problem for its configured 5000 steps on a 128x96x160 grid
    (the full grid's oracle would take most of an hour).  A and C meet the
    FP32 target.  B does not, and no FP32 evaluation of the step can: B
    (about 0.1) changes by less than half its FP32 spacing per step over
    much of the grid, so those increments are rounded away, and a plain
    numpy FP32 evaluation of the same step lands on the same error against
    FP64 (rel-L2 3.3e-5, max-abs 7.6e-6 -- the max-abs bound holds).  B's
    rel-L2 is held to three times that floor."""
    w = W.make_workload("front384", shape=(160, 96, 128))
    got, plan = run_autotuned(w, w.steps)
    ref = oracle.run(w.spec, w.fields, w.steps)
    check_fp32("front 128x96x160", w, w.steps, got, ref, plan, tol=[TOL, 1e-4, TOL])


@pytest.mark.timeout(900)
def test_pollutant_configured_steps_reduced_grid():
    """The pollutant problem for its configured 3000 steps on a 128x128x64
    grid with its 64 seeded sources (the full grid is a recorded run)."""
    w = W.make_workload("pollutant512", shape=(64, 128, 128))
    got, plan = run_autotuned(w, w.steps)
    ref = oracle.run(w.spec, w.fields, w.steps)
    check_fp32("pollutant 128x128x64", w, w.steps, got, ref, plan)
