"""GPU tests of stochastic rounding of BF16 stores.

The rounding decisions are predicted cell by cell with the oracle side's own
Philox-2x32-10 and rounding definition (bit-exact, every plan, two steps so
the step counter is checked too); a slow decay that round-to-nearest BF16
freezes is followed by stochastic rounding in the mean; plans, graphs and
repeated runs give the same bits; the refusals hold.
"""
import numpy as np
import pytest

import oracle
from oracle.stochastic import bf16_stochastic, random16
from paper_1004_0480_amd import rd
from paper_1004_0480_amd import workloads as W
from paper_1004_0480_amd.workloads import MIRROR, ModelSpec, uniform_bc
from test_gpu_parity import compiled_plans, gpu_run, rel_l2

pytestmark = pytest.mark.gpu


def decay_spec(shape, lam, dt):
    """One pollutant with decay only: c' = c - dt lam c."""
    return ModelSpec("pollutant", 1, dt, 1.0, [[0.0] * 3], uniform_bc(1, MIRROR), {"decay": lam, "kab": 0.0},
                     wind=np.zeros(shape[0]))


def dense_index(shape):
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (k * ny + j) * nx + i


@pytest.mark.parametrize("shape", [(5, 7, 70), (6, 9, 256)])
def test_stochastic_bits_are_the_counter_generators(shape):
    """Decay by exactly 2^-10 per step from 1.0: the FP32 results are exact,
    so every stored bit follows from the generator: the cell rounds up when
    its 16 random bits reach 2^16 minus the discarded bits."""
    seed = 20240611
    spec = decay_spec(shape, 2.0**-5, 2.0**-5)
    c0 = np.ones(shape)
    idx = dense_index(shape)
    x1 = np.full(shape, 1.0 - 2.0**-10)
    y1 = bf16_stochastic(x1.astype(np.float32), random16(idx, 0, seed, 0)).astype(np.float64)
    x2 = y1 - y1 * 2.0**-10
    assert np.array_equal(x2.astype(np.float32).astype(np.float64), x2)
    y2 = bf16_stochastic(x2.astype(np.float32), random16(idx, 1, seed, 0)).astype(np.float64)
    assert 0.6 < np.mean(y1 == 1.0) < 0.9                       # P(up) = 3/4
    w = W.Workload("decay", shape, spec, [c0], 2, 0)
    for plan in compiled_plans(w, storage="bf16", czs=(0, 4)):
        for steps, want in ((1, y1), (2, y2)):
            g = rd.Grid(shape, 1, 1.0, "bf16")
            g.set_model(spec)
            g.set_rounding("stochastic", seed)
            g.set_plan(**plan)
            g.write(0, c0)
            g.step(steps)
            got = g.read(0)
            g.close()
            assert np.array_equal(got, want), (plan, steps, int(np.sum(got != want)))


def test_stochastic_rounding_follows_a_slow_decay():
    """dt lam = 1e-3: round-to-nearest BF16 keeps 1.0 for ever (the step is
    below half a unit), stochastic rounding tracks the FP64 decay in the mean."""
    shape = (64, 64, 64)
    spec = decay_spec(shape, 1e-3, 1.0)
    n = 500
    exact = oracle.run(spec, [np.ones(shape)], n)[0]
    means = {}
    for mode in ("nearest", "stochastic"):
        g = rd.Grid(shape, 1, 1.0, "bf16")
        g.set_model(spec)
        g.set_rounding(mode, 7)
        g.write(0, np.ones(shape))
        g.step(n)
        means[mode] = float(np.mean(g.read(0)))
        g.close()
    target = float(np.mean(exact))
    assert abs(target - 0.999**n) < 1e-12
    assert means["nearest"] == 1.0
    assert abs(means["stochastic"] - target) < 2e-3, (means, target)


def test_stochastic_plans_graphs_and_repeats():
    """Brusselator with stochastic BF16 stores: every plan and a graph replay
    give the same bits, the same seed repeats them, another seed does not,
    and the fields stay at the BF16 level of the FP64 oracle."""
    import torch
    w = W.make_workload("brusselator256", shape=(6, 10, 256))
    steps = 6

    def run(plan=None, seed=3, chunk=0):
        g = rd.Grid(w.shape, 2, 1.0, "bf16", stream=torch.cuda.Stream() if chunk else None)
        g.set_model(w.spec)
        g.set_rounding("stochastic", seed)
        if plan:
            g.set_plan(**plan)
        if chunk:
            g.set_plan(graph_chunk=chunk)
        for s in range(2):
            g.write(s, w.fields[s])
        g.step(steps)
        out = g.read_all()
        g.close()
        return out

    base = run()
    for plan in compiled_plans(w, storage="bf16", czs=(0, 4)):
        got = run(plan)
        assert all(np.array_equal(a, b) for a, b in zip(got, base)), plan
    assert all(np.array_equal(a, b) for a, b in zip(run(chunk=2), base))
    assert all(np.array_equal(a, b) for a, b in zip(run(), base))
    assert not all(np.array_equal(a, b) for a, b in zip(run(seed=4), base))
    ref = oracle.run(w.spec, w.fields, steps)
    for s in range(2):
        assert rel_l2(base[s], ref[s]) <= 1e-2


@pytest.mark.parametrize("shape", [(6, 10, 256), (5, 9, 200), (5, 6, 130)])
def test_stochastic_front_every_plan_same_bits(shape):
    """Three-species front model with stochastic BF16 stores: the one-pass
    kernel (whose lane pairs share the generator's calls when the rows are a
    multiple of four long) stores the same bits as every other plan, which
    store through the general per-cell draw."""
    w = W.make_workload("front384", shape=shape)
    steps = 3

    def run(plan=None):
        g = rd.Grid(w.shape, 3, w.spec.h, "bf16")
        g.set_model(w.spec)
        g.set_rounding("stochastic", 11)
        if plan:
            g.set_plan(**plan)
        for s in range(3):
            g.write(s, w.fields[s])
        g.step(steps)
        out = g.read_all()
        g.close()
        return out

    base = run(dict(kernel="direct"))
    plans = compiled_plans(w, storage="bf16", czs=(0, 4))
    assert any(p["kernel"] == "fused" for p in plans)
    for plan in plans:
        got = run(plan)
        assert all(np.array_equal(a, b) for a, b in zip(got, base)), plan


def test_stochastic_rounding_refusals():
    import torch
    shape = (8, 8, 64)
    spec = decay_spec(shape, 1e-3, 1.0)
    g = rd.Grid(shape, 1, 1.0, "f32")
    with pytest.raises(rd.RDError) as ei:
        g.set_rounding("stochastic", 1)
    assert ei.value.code == rd.EINVAL
    g.close()
    g = rd.Grid(shape, 1, 1.0, "bf16")
    g.set_rounding("stochastic", 1)
    rk = spec.copy()
    rk.integrator = "rk2"
    with pytest.raises(rd.RDError) as ei:
        g.set_model(rk)
    assert ei.value.code == rd.EINVAL
    g.close()
    stream = torch.cuda.Stream()
    b = rd.Batch(2, 1 << 30, "bf16", stream=stream)
    d = W.diffusion_spec()
    g = rd.Grid(shape, 1, 1.0, "bf16", stream=stream)
    g.set_model(d)
    g.set_rounding("stochastic", 1)
    with pytest.raises(rd.RDError) as ei:
        b.add(g, 3)
    assert ei.value.code == rd.EINVAL
    b.close()
    g.close()
