"""GPU parity for the strong-stability-preserving Runge-Kutta steps (order 2,
Heun, and order 3, Shu-Osher) built from the Euler kernels: every plan the
library accepts against the FP64 oracle's Runge-Kutta run and bit for bit
against each other, graph replays and split calls, and the refusals.
"""
import numpy as np
import pytest

import oracle
from paper_1004_0480_amd import rd
from paper_1004_0480_amd import workloads as W
from paper_1004_0480_amd.workloads import GHOST, HELD, MIRROR, PERIODIC, ModelSpec, uniform_bc
from test_gpu_parity import TOL, bc_spec, compiled_plans, gpu_run, rel_l2

pytestmark = pytest.mark.gpu


def case(name, integrator):
    rng = np.random.default_rng(sum(map(ord, name + integrator)))
    if name.startswith("faces"):
        nx = int(name[5:])
        shape = (8, 9, nx)
        faces = [(HELD, 1.0), (GHOST, -0.5), (PERIODIC, 0), (PERIODIC, 0), (GHOST, 2.0), (HELD, -1.0)]
        spec = bc_spec(2, faces, K=(1.0, 0.5, 0.25), dt=0.1)
        fields = [rng.uniform(0, 1, shape) for _ in range(2)]
        w = W.Workload(name, shape, spec, fields, 6, 0)
    elif name == "bruss19":
        w = W.make_workload("brusselator256", shape=(6, 10, 256))
        w.spec.stencil = 19
    elif name == "front":
        w = W.make_workload("front384", shape=(9, 10, 70))
        w.fields = [f.astype(np.float32).astype(np.float64) for f in w.fields]
        w.fields[2] = rng.uniform(-1, 1, w.shape)
    elif name == "pollutant":
        w = W.make_workload("pollutant512", shape=(8, 10, 128))
        w.fields = [rng.uniform(0, 1, w.shape) for _ in range(4)]
    elif name == "turing19":
        shape = (7, 9, 192)
        spec = W.turing_spec(stencil=19)
        w = W.Workload(name, shape, spec, [1.0 + rng.uniform(-0.05, 0.05, shape) for _ in range(2)], 6, 0)
    else:
        raise KeyError(name)
    w.spec.integrator = integrator
    return w


@pytest.mark.parametrize("integrator", ["rk2", "rk3"])
@pytest.mark.parametrize("name", ["faces70", "faces256", "bruss19", "front", "pollutant", "turing19"])
def test_rk_every_plan(name, integrator):
    w = case(name, integrator)
    steps = 5
    ref = oracle.run(w.spec, w.fields, steps)
    plans = compiled_plans(w, czs=(0, 4))
    assert not any(p["kernel"] == "lds2" for p in plans)
    base = None
    for plan in plans:
        got, _ = gpu_run(w, steps, plan=plan)
        if base is None:
            base = got
            for s in range(w.spec.ns):
                e = rel_l2(got[s], ref[s])
                assert e <= TOL, (name, integrator, s, e)
            continue
        for s in range(w.spec.ns):
            assert np.array_equal(got[s], base[s]), (name, integrator, plan, s)


@pytest.mark.parametrize("integrator", ["rk2", "rk3"])
def test_rk_graphs_and_split_calls(integrator):
    """Graph replays of chunks of Runge-Kutta steps and split calls give the
    bits of eager steps; the autotuner leaves the state as it was."""
    import torch
    w = case("faces256", integrator)
    n = 11

    def run(split, chunk=0, tune=False):
        g = rd.Grid(w.shape, 2, w.spec.h, "f32", stream=torch.cuda.Stream() if chunk else None)
        g.set_model(w.spec)
        for s in range(2):
            g.write(s, w.fields[s])
        if tune:
            g.autotune(2)
        g.set_plan(graph_chunk=chunk)
        for k in split:
            g.step(k)
        out = g.read_all()
        g.close()
        return out

    eager = run([n])
    ref = oracle.run(w.spec, w.fields, n)
    for s in range(2):
        assert rel_l2(eager[s], ref[s]) <= TOL
    for got in (run([4, 7]), run([n], chunk=4), run([3, 8], chunk=2), run([n], tune=True)):
        for s in range(2):
            assert np.array_equal(got[s], eager[s])


def test_rk_bf16_storage_runs_close():
    """BF16 storage rounds every stage; the error stays at the BF16 level."""
    w = case("faces256", "rk2")
    got, _ = gpu_run(w, 5, storage="bf16")
    ref = oracle.run(w.spec, w.fields, 5)
    for s in range(2):
        assert rel_l2(got[s], ref[s]) <= 1e-2


def test_rk_refusals():
    import torch
    shape = (8, 8, 256)
    spec = bc_spec(1, [(MIRROR, 0)] * 6, K=(1.0, 1.0, 1.0), dt=0.1)
    spec.integrator = "rk2"
    g = rd.Grid(shape, 1, 1.0)
    g.set_model(spec)
    with pytest.raises(rd.RDError) as ei:
        g.set_plan(kernel="lds2", vx=4, ry=4, waves=8, prefetch=6)
    assert ei.value.code == rd.EINVAL
    stream = torch.cuda.Stream()
    b = rd.Batch(2, 1 << 30, "f32", stream=stream)
    g2 = rd.Grid(shape, 1, 1.0, stream=stream)
    g2.set_model(spec)
    with pytest.raises(rd.RDError) as ei:
        b.add(g2, 3)
    assert ei.value.code == rd.EINVAL
    b.close()
    g2.close()
    a = ModelSpec("atmos", 1, 0.1, 1.0, [[0.1] * 3], uniform_bc(1, MIRROR),
                  {"ux": 1.0, "uy": 0.0, "uz": 1.0, "uz_period": 2.0}, integrator="rk3")
    with pytest.raises(rd.RDError) as ei:
        g.set_model(a)
    assert ei.value.code == rd.EINVAL
    g.close()
