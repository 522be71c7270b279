"""Served batch on the GPU: every result equals the same request run alone
(bitwise), and a served result matches the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1004_0480_amd import rd
from paper_1004_0480_amd import serve as S
from paper_1004_0480_amd import workloads as W

pytestmark = pytest.mark.gpu


def alone(req, storage):
    g = rd.Grid((req.edge,) * 3, 2 if req.model == "brusselator" else 1, 1.0, storage)
    g.set_model(W.request_spec(req))
    init = W.request_fields_device(req)
    for s, f in enumerate(init):
        g.write(s, f)
    g.step(req.steps)
    out = g.read_all(np.float32)
    g.close()
    return out, [f.cpu().numpy().astype(np.float64) for f in init]


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_served_results_equal_alone(storage):
    tr = W.make_trace(24, seed=11, edges=(32, 48, 64), min_steps=20, max_steps=90)
    arr = S.poisson_arrivals(tr, 300.0)
    ex = S.GpuExecutor(storage, max_resident=12, hbm_budget=1 << 34)
    rep = S.serve(tr, arr, ex, 12, 1 << 34, chunk=16, keep_results=True)
    ex.close()
    assert len(rep.completions) == len(tr)
    print(storage, rep.summary())
    overlapped = sum(1 for c in rep.completions
                     if any(o.admitted < c.admitted < o.finished for o in rep.completions if o is not c))
    assert overlapped > 0                      # requests joined while others were on the GPU
    for i, req in enumerate(tr):
        a, _ = alone(req, storage)
        for s in range(len(a)):
            assert np.array_equal(a[s], rep.results[i][s]), (i, req, s)


def test_served_result_matches_oracle():
    req = W.Request(0, 0.0, 48, "brusselator", 60, 12345)
    tr = [req, W.Request(1, 0.0, 32, "diffusion", 40, 777)]
    ex = S.GpuExecutor("f32", max_resident=4, hbm_budget=1 << 32)
    rep = S.serve(tr, [0.0, 0.0], ex, 4, 1 << 32, chunk=25, keep_results=True)
    ex.close()
    _, init = alone(req, "f32")
    ref = oracle.run(W.request_spec(req), init, req.steps)
    for s in range(2):
        got = rep.results[0][s].astype(np.float64)
        e = np.linalg.norm(got - ref[s]) / np.linalg.norm(ref[s])
        assert e <= 1e-5, e
