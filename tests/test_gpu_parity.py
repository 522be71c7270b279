"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

FP32 fields must match the oracle to relative L2 <= 1e-5 per species after
the stated steps; every kernel plan must give bitwise-identical fields; BF16
and FP16 storage must lie within one unit in the last place of the oracle's
step rounded to the storage type.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1004_0480_amd import rd
from paper_1004_0480_amd import workloads as W
from paper_1004_0480_amd.workloads import GHOST, HELD, MIRROR, PERIODIC, ModelSpec

pytestmark = pytest.mark.gpu

TOL = 1e-5          # FP32 rel-L2 bound per species against the FP64 oracle

# candidate (vx, ry, waves, prefetch) z-march shapes and (vx, ry, waves, cz)
# slab shapes; the library rejects the ones it did not compile for a model
TILE_SHAPES = [(4, 1, 4, 1), (4, 1, 4, 2), (2, 2, 4, 2), (2, 1, 4, 2), (4, 2, 4, 1), (1, 4, 4, 2),
               (2, 1, 4, 1)]
# LDS-ring shapes (cells per lane = 4 * 256-cell chunks, rows per workgroup,
# computing waves, ring slots); only rows of exactly 64 * vx cells take them
LDS_SHAPES = [(4, 8, 4, 7), (4, 8, 8, 7), (8, 8, 4, 6), (8, 4, 4, 6), (8, 8, 8, 6), (8, 4, 4, 7),
              (8, 8, 8, 7), (4, 12, 6, 5), (8, 12, 6, 5), (8, 6, 6, 5), (4, 4, 4, 6), (8, 2, 2, 5)]
# two-steps-per-launch shapes (same fields)
LDS2_SHAPES = [(4, 4, 8, 6), (8, 4, 8, 6), (4, 8, 8, 5), (8, 6, 6, 4), (4, 6, 12, 4), (8, 6, 12, 4),
               (8, 4, 12, 6), (4, 4, 12, 6)]
# one-pass front shapes (rows per workgroup, update waves, chemical-potential
# waves, ring slots)
FCH_SHAPES = [(8, 8, 5, 7), (4, 4, 3, 7), (4, 4, 3, 6), (2, 2, 2, 7), (4, 4, 2, 7), (8, 8, 4, 8), (16, 8, 6, 7),
              (4, 4, 3, 9), (8, 8, 5, 6), (4, 4, 3, 5), (4, 4, 2, 5), (8, 8, 5, 5)]
TR_SHAPES = [(8, 8, 6), (4, 4, 7), (8, 4, 6), (4, 4, 6), (8, 8, 5), (16, 8, 5), (8, 8, 4), (6, 6, 5),
             (16, 8, 6), (16, 8, 7)]
BLOCK_SHAPES = [(4, 1, 4, 2), (4, 1, 4, 4), (4, 2, 4, 2), (4, 2, 4, 4), (4, 1, 4, 8), (2, 2, 4, 4),
                (2, 1, 4, 4), (4, 2, 1, 2), (4, 1, 1, 2), (4, 2, 1, 4), (4, 4, 1, 2), (4, 2, 2, 2),
                (4, 3, 1, 2)]


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu_run(w, steps, storage="f32", plan=None, fields=None):
    g = rd.Grid(w.shape, w.spec.ns, w.spec.h, storage)
    g.set_model(w.spec)
    if plan:
        g.set_plan(**plan)
    for s, f in enumerate(fields if fields is not None else w.fields):
        g.write(s, f)
    g.step(steps)
    out = g.read_all()
    used = g.plan()
    g.close()
    return out, used


def compiled_plans(w, storage="f32", czs=(0, 8)):
    """Every tiled plan the library accepts for this model, plus direct."""
    plans = [dict(kernel="direct")]
    g = rd.Grid(w.shape, w.spec.ns, w.spec.h, storage)
    g.set_model(w.spec)
    cands = [dict(kernel="tiled", vx=vx, ry=ry, waves=wv, cz=cz, prefetch=pf)
             for vx, ry, wv, pf in TILE_SHAPES for cz in czs]
    cands += [dict(kernel="block", vx=vx, ry=ry, waves=wv, cz=cz, order=o)
              for vx, ry, wv, cz in BLOCK_SHAPES for o in (0, 1)]
    cands += [dict(kernel="lds", vx=vx, ry=by, waves=wc, prefetch=d, cz=cz, order=o)
              for vx, by, wc, d in LDS_SHAPES for cz in czs for o in (0, 1)]
    cands += [dict(kernel="lds2", vx=vx, ry=by, waves=wc, prefetch=d, cz=cz, order=o)
              for vx, by, wc, d in LDS2_SHAPES for cz in czs for o in (0, 1)]
    cands += [dict(kernel="fused", vx=wm, ry=by, waves=wu, prefetch=d, cz=cz, order=o)
              for by, wu, wm, d in FCH_SHAPES for cz in czs for o in (0, 1)]
    cands += [dict(kernel="tring", vx=2, ry=by, waves=wc, prefetch=d, cz=cz, order=o)
              for by, wc, d in TR_SHAPES for cz in czs for o in (0, 1)]
    for p in cands:
        try:
            g.set_plan(**p)
        except rd.RDError:
            continue
        plans.append(p)
    g.close()
    return plans


def check_parity(w, steps, tol=TOL, storage="f32", plan=None, label=""):
    got, used = gpu_run(w, steps, storage, plan)
    ref = oracle.run(w.spec, w.fields, steps)
    for s in range(w.spec.ns):
        e = rel_l2(got[s], ref[s])
        m = float(np.max(np.abs(got[s] - ref[s])))
        print("%s %s species %d: rel-L2 %.3e max-abs %.3e plan %s" % (label or w.name, w.shape, s, e, m, used))
        assert e <= tol, (label, s, e)
    return got, ref


# ------------------------------------------------------------ workloads

@pytest.mark.parametrize("plan", [None, dict(kernel="direct")])
def test_diffusion64_full_run(plan):
    """64^3 no-flux diffusion, 100 steps: the whole configured run."""
    w = W.make_workload("diffusion64")
    check_parity(w, w.steps, plan=plan)


def test_quadratic_field_bitwise_on_interior():
    """Integer quadratic, dyadic coefficients: FP32 is exact, so the GPU and
    the oracle agree bit for bit on interior cells (across several tiles)."""
    shape = (11, 37, 300)
    k, j, i = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    c0 = (3 * i**2 - 2 * j**2 + 5 * k**2 + 4 * i - 7 * j + 2 * k + 11).astype(float)
    spec = ModelSpec("diffusion", 1, 0.0625, 1.0, [[2.0, 3.0, 0.5]], W.uniform_bc(1, MIRROR))
    w = W.Workload("quadratic", shape, spec, [c0], 1, 0)
    ref = oracle.run(spec, [c0], 1)[0]
    inner = (slice(1, -1),) * 3
    for plan in compiled_plans(w, czs=(0, 4)):
        got, _ = gpu_run(w, 1, plan=plan)
        assert np.array_equal(got[0][inner], ref[inner]), plan


def test_brusselator_ragged_parity():
    w = W.make_workload("brusselator256", shape=(23, 37, 70))
    check_parity(w, 50)


def test_brusselator_long_run():
    """2000 steps (the configured length) on a 64^3 periodic grid."""
    w = W.make_workload("brusselator256", shape=(64, 64, 64))
    check_parity(w, 2000)


def test_brusselator_full_size_default_plan():
    """256^3 in the plan the benchmark uses (autotuned), 10 steps."""
    w = W.make_workload("brusselator256")
    g = rd.Grid.from_workload(w)
    g.autotune(5)
    g.step(10)
    got = g.read_all()
    plan = g.plan()
    g.close()
    ref = oracle.run(w.spec, w.fields, 10)
    for s in range(2):
        e = rel_l2(got[s], ref[s])
        print("brusselator256 full size species %d rel-L2 %.3e plan %s" % (s, e, plan))
        assert e <= TOL


def test_front_parity():
    w = W.make_workload("front384", shape=(48, 36, 40))
    check_parity(w, 200)


def test_front_chemical_potential_pass():
    """The first Laplacian pass alone, from an FP32-exact state."""
    w = W.make_workload("front384", shape=(20, 24, 70))
    rng = np.random.default_rng(4)
    fields = [f.astype(np.float32).astype(np.float64) for f in w.fields]
    fields[2] = rng.uniform(-1.2, 1.2, w.shape).astype(np.float32).astype(np.float64)
    g = rd.Grid(w.shape, 3, 1.0)
    g.set_model(w.spec)
    for s in range(3):
        g.write(s, fields[s])
    mu = g.chemical_potential().astype(np.float64)
    g.close()
    ref = oracle.chemical_potential(w.spec, fields)
    assert np.max(np.abs(mu - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("nx", [70, 128])
def test_front_held_and_ghost_corners_every_plan(nx):
    """C held on some faces and fixed ghosts on others: the chemical
    potential (not held) is evaluated on held cells, where a ghost beyond a
    face must win over a held layer of another axis.  Every plan matches the
    oracle's first pass and its steps."""
    w = W.make_workload("front384", shape=(9, 10, nx))
    spec = w.spec
    spec.bc[2] = [(HELD, 0.3), (GHOST, 0.1), (GHOST, -0.2), (HELD, 0.4), (HELD, 0.5), (GHOST, 0.0)]
    spec.bc[1] = [(GHOST, 0.2), (HELD, 0.6), (MIRROR, 0), (GHOST, 0.3), (MIRROR, 0), (HELD, 0.1)]
    rng = np.random.default_rng(11)
    fields = [f.astype(np.float32).astype(np.float64) for f in w.fields]
    fields[2] = rng.uniform(-1.0, 1.0, w.shape).astype(np.float32).astype(np.float64)
    w = W.Workload("front_corners", w.shape, spec, fields, 4, 0)
    mu_ref = oracle.chemical_potential(spec, fields)
    ref = oracle.run(spec, fields, 4)
    base = None
    for plan in compiled_plans(w, czs=(0, 4)):
        g = rd.Grid(w.shape, 3, 1.0)
        g.set_model(spec)
        g.set_plan(**plan)
        for s in range(3):
            g.write(s, fields[s])
        mu = g.chemical_potential().astype(np.float64)
        g.close()
        assert np.max(np.abs(mu - mu_ref)) <= 1e-5 * max(1.0, np.max(np.abs(mu_ref))), plan
        got, _ = gpu_run(w, 4, plan=plan)
        if base is None:
            base = got
            for s in range(3):
                assert rel_l2(got[s], ref[s]) <= TOL, (plan, s)
        for s in range(3):
            assert np.array_equal(got[s], base[s]), (plan, s)


def test_front_conserves_b_plus_c_on_gpu():
    """sum(B + C) is invariant (B, C no-flux; A+B->C moves mass between them);
    the GPU's FP64 reductions see only FP32 rounding drift."""
    w = W.make_workload("front384", shape=(40, 32, 48))
    g = rd.Grid.from_workload(w)
    m0 = g.reduce(1)[0] + g.reduce(2)[0]
    g.step(500)
    m1 = g.reduce(1)[0] + g.reduce(2)[0]
    g.close()
    drift = abs(m1 - m0) / abs(m0)
    print("front sum(B+C) relative drift after 500 FP32 steps: %.3e" % drift)
    assert drift < 1e-5


def test_pollutant_parity():
    w = W.make_workload("pollutant512", shape=(24, 40, 96))
    check_parity(w, 300)


def test_pass_structure():
    """One launch per step, or two: the front model's chemical-potential pass
    (one launch with the one-pass plan, the default), and more than two
    pollutants split into the coupled pair and the rest."""
    expect = {"brusselator256": 1, "diffusion64": 1, "front384": 1, "pollutant512": 2}
    for name, n in expect.items():
        w = W.make_workload(name, shape=(6, 7, 9))
        g = rd.Grid.from_workload(w)
        assert g.passes() == n, name
        if name == "front384":
            assert g.plan()["kernel"] == rd.KERNEL["fused"]
            g.set_plan(kernel="direct")
            assert g.passes() == 2
        g.close()
    for ns, n in ((1, 1), (2, 1), (3, 2)):
        shape = (6, 7, 9)
        spec = W.pollutant_spec(shape, 1, ns=ns)
        g = rd.Grid(shape, ns, 1.0)
        g.set_model(spec)
        assert g.passes() == n, ns
        g.close()


@pytest.mark.parametrize("ns", [1, 2, 3])
def test_pollutant_species_groups_parity(ns):
    """Fewer pollutants than the configured four: one pass (one or two
    species) or two (the coupled pair, then a single species whose sources
    are found by their global species index)."""
    shape = (14, 20, 72)
    spec = W.pollutant_spec(shape, 5, ns=ns, nsrc=40, rate=50.0)
    rng = np.random.default_rng(ns)
    fields = [rng.uniform(0, 1, shape) for _ in range(ns)]
    w = W.Workload("pollutant_ns%d" % ns, shape, spec, fields, 80, 5)
    check_parity(w, 80)


def test_pollutant_ragged_multi_tile():
    w = W.make_workload("pollutant512", shape=(17, 21, 300))
    check_parity(w, 60)


# --------------------------------------------------------- plans agree

@pytest.mark.parametrize("name,shape,steps", [
    ("diffusion64", (19, 27, 130), 7),
    ("brusselator256", (13, 22, 200), 6),
    ("front384", (14, 18, 150), 5),
    ("pollutant512", (12, 19, 140), 6),
])
def test_every_plan_bitwise_identical(name, shape, steps):
    w = W.make_workload(name, shape=shape)
    base = None
    for plan in compiled_plans(w, czs=(0, 5)):
        got, _ = gpu_run(w, steps, plan=plan)
        if base is None:
            base = got
            continue
        for s in range(w.spec.ns):
            assert np.array_equal(got[s], base[s]), (name, plan, s)


# ------------------------------------------------ one-pass front step (P9)

def front_case(case):
    """Front-model grids for the one-pass plan: ragged and whole 128-cell
    tiles, one-cell last tiles, every face kind on C (mu stays mirrored),
    held and fixed faces on A and B, periodic x (whole tiles)."""
    base = {"nx70": (9, 10, 70), "nx129": (7, 11, 129), "nx200": (8, 13, 200), "nx256p": (7, 9, 256),
            "nx384": (6, 17, 384), "nx128p": (10, 8, 128), "nx257": (5, 9, 257)}[case]
    w = W.make_workload("front384", shape=base)
    spec = w.spec
    rng = np.random.default_rng(sum(base))
    if case in ("nx70", "nx200", "nx257"):
        spec.bc[2] = [(HELD, 0.3), (GHOST, 0.1), (GHOST, -0.2), (HELD, 0.4), (HELD, 0.5), (GHOST, 0.0)]
        spec.bc[1] = [(GHOST, 0.2), (HELD, 0.6), (MIRROR, 0), (GHOST, 0.3), (MIRROR, 0), (HELD, 0.1)]
    elif case == "nx129":
        spec.bc[2] = [(MIRROR, 0), (HELD, -0.25), (MIRROR, 0), (GHOST, 0.5), (GHOST, -0.5), (MIRROR, 0)]
        spec.bc[0] = [(HELD, 1.0), (GHOST, 0.0), (PERIODIC, 0), (PERIODIC, 0), (MIRROR, 0), (MIRROR, 0)]
    elif case in ("nx256p", "nx128p"):
        for s in range(3):
            spec.bc[s][0] = spec.bc[s][1] = (PERIODIC, 0.0)
        spec.bc[2][2] = spec.bc[2][3] = (PERIODIC, 0.0)
        spec.bc[2][4] = spec.bc[2][5] = (PERIODIC, 0.0)
    fields = [f.astype(np.float32).astype(np.float64) for f in w.fields]
    fields[0] = rng.uniform(0.0, 1.0, base).astype(np.float32).astype(np.float64)
    fields[2] = rng.uniform(-1.0, 1.0, base).astype(np.float32).astype(np.float64)
    return W.Workload("front_" + case, base, spec, fields, 5, 0)


@pytest.mark.parametrize("case", ["nx70", "nx129", "nx200", "nx256p", "nx384", "nx128p", "nx257"])
def test_front_one_pass_bitwise_equals_two_pass(case):
    """The one-pass front step computes mu in LDS instead of an array, with
    the same arithmetic: every one-pass shape gives the bits of the two-pass
    direct plan, which matches the FP64 oracle."""
    w = front_case(case)
    steps = 5
    ref = oracle.run(w.spec, w.fields, steps)
    two, _ = gpu_run(w, steps, plan=dict(kernel="direct"))
    for s in range(3):
        assert rel_l2(two[s], ref[s]) <= TOL, (case, s)
    plans = [p for p in compiled_plans(w, czs=(0, 1, 3)) if p["kernel"] == "fused"]
    assert plans, case
    for plan in plans:
        got, _ = gpu_run(w, steps, plan=plan)
        for s in range(3):
            assert np.array_equal(got[s], two[s]), (case, plan, s)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_front_one_pass_reduced_storage_and_rk(storage):
    """2-byte storage and the Runge-Kutta stages on the one-pass plan: the
    same bits as the two-pass direct plan."""
    w = front_case("nx200")
    for integ in ("euler", "rk2", "rk3"):
        if integ != "euler" and storage == "f16":
            continue
        w.spec.integrator = integ
        two, _ = gpu_run(w, 4, storage=storage, plan=dict(kernel="direct"))
        plans = [p for p in compiled_plans(w, storage=storage, czs=(0, 3)) if p["kernel"] == "fused"]
        assert plans
        for plan in plans:
            got, _ = gpu_run(w, 4, storage=storage, plan=plan)
            for s in range(3):
                assert np.array_equal(got[s], two[s]), (storage, integ, plan, s)
    w.spec.integrator = "euler"


def test_front_one_pass_refusals():
    """The one-pass plan takes the 7-point front model only, and a periodic x
    axis of C only for nx <= 128 or a multiple of 128."""
    w = W.make_workload("brusselator256", shape=(6, 8, 70))
    g = rd.Grid.from_workload(w)
    with pytest.raises(rd.RDError):
        g.set_plan(kernel="fused", vx=3, ry=4, waves=4, prefetch=7)
    g.close()
    w = front_case("nx200")
    for s in range(3):
        w.spec.bc[s][0] = w.spec.bc[s][1] = (PERIODIC, 0.0)
    g = rd.Grid.from_workload(w)
    with pytest.raises(rd.RDError):
        g.set_plan(kernel="fused", vx=3, ry=4, waves=4, prefetch=7)
    g.close()
    w19 = as19(front_case("nx70"))
    g = rd.Grid.from_workload(w19)
    with pytest.raises(rd.RDError):
        g.set_plan(kernel="fused", vx=3, ry=4, waves=4, prefetch=7)
    g.close()


# ---------------------------------------------------- storage precisions

def round_bf16(x):
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def round_f16(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


def ulp(x, storage):
    a = np.abs(x)
    if storage == "bf16":
        e = np.floor(np.log2(np.maximum(a, 1e-30)))
        return 2.0 ** (e - 7)
    return np.spacing(np.maximum(a, 6.1e-5).astype(np.float16)).astype(np.float64)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
@pytest.mark.parametrize("name,shape", [("brusselator256", (9, 14, 80)),
                                        ("front384", (10, 12, 70)),
                                        ("diffusion64", (16, 16, 130))])
def test_reduced_storage_single_step_within_one_ulp(storage, name, shape):
    w = W.make_workload(name, shape=shape)
    rnd = round_bf16 if storage == "bf16" else round_f16
    start = [rnd(f) for f in w.fields]
    got, _ = gpu_run(w, 1, storage=storage, fields=start)
    ref = oracle.run(w.spec, start, 1)
    for s in range(w.spec.ns):
        expect = rnd(ref[s])
        assert np.all(np.abs(got[s] - expect) <= ulp(expect, storage) * 1.0001), (storage, name, s)


def test_bf16_front_error_reported():
    """BF16 storage error against FP64 is reported (not a target)."""
    w = W.make_workload("front384", shape=(32, 24, 40))
    steps = 200
    got, _ = gpu_run(w, steps, storage="bf16")
    ref = oracle.run(w.spec, w.fields, steps)
    for s in range(3):
        e = rel_l2(got[s], ref[s])
        print("front bf16 storage, %d steps, species %d: rel-L2 %.3e max-abs %.3e"
              % (steps, s, e, np.max(np.abs(got[s] - ref[s]))))
        assert np.all(np.isfinite(got[s])) and e < 1.0


# ------------------------------------------------------------ reductions

@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_fp64_reduction_matches_oracle(storage):
    w = W.make_workload("brusselator256", shape=(30, 41, 77))
    g = rd.Grid.from_workload(w, storage=storage)
    g.step(3)
    for s in range(2):
        f = g.read(s)
        m, e = g.reduce(s)
        mo, eo = oracle.reduce(f, 1.0)
        assert abs(m - mo) <= 1e-12 * abs(mo) and abs(e - eo) <= 1e-12 * abs(eo)
    g.close()


def test_nonfinite_field_detected():
    w = W.make_workload("diffusion64", shape=(8, 8, 8))
    f = w.fields[0].copy()
    f[3, 4, 5] = np.nan
    g = rd.Grid(w.shape, 1)
    g.set_model(w.spec)
    g.write(0, f)
    with pytest.raises(rd.RDError) as ei:
        g.reduce(0)
    assert ei.value.code == rd.ENONFINITE
    g.close()


# ------------------------------------------------------ host-side paths

def test_checkpoint_round_trip_is_bitwise():
    w = W.make_workload("brusselator256", shape=(16, 20, 90))
    a, _ = gpu_run(w, 30)
    g = rd.Grid.from_workload(w)
    g.step(13)
    saved = g.read_all()
    g.close()
    g2 = rd.Grid(w.shape, 2)
    g2.set_model(w.spec)
    for s in range(2):
        g2.write(s, saved[s])
    g2.step(17)
    b = g2.read_all()
    g2.close()
    for s in range(2):
        assert np.array_equal(a[s], b[s])


def test_graph_replay_matches_eager():
    import torch
    stream = torch.cuda.Stream()
    w = W.make_workload("front384", shape=(20, 24, 64))
    eager, _ = gpu_run(w, 37)
    g = rd.Grid(w.shape, 3, 1.0, "f32", stream=stream)
    g.set_model(w.spec)
    g.set_plan(graph_chunk=6)
    for s, f in enumerate(w.fields):
        g.write(s, f)
    g.step(20)
    g.step(17)
    got = g.read_all()
    g.close()
    for s in range(3):
        assert np.array_equal(got[s], eager[s])


def test_autotune_keeps_state_and_plans_agree():
    w = W.make_workload("diffusion64", shape=(40, 48, 200))
    g = rd.Grid.from_workload(w)
    before = g.read(0)
    plan = g.autotune(3)
    assert np.array_equal(g.read(0), before)
    g.set_plan(**plan)
    g.step(9)
    got = g.read(0)
    g.close()
    ref, _ = gpu_run(w, 9, plan=dict(kernel="direct"))
    assert np.array_equal(got, ref[0])


def test_copy_probe_copies():
    import torch
    src = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    rd.copy_probe(dst.data_ptr(), src.data_ptr(), src.numel() * 4)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


# --------------------------------------------------------------- edges

def bc_spec(ns, faces, K=(1.0, 0.5, 0.25), dt=0.1):
    return ModelSpec("diffusion", ns, dt, 1.0, [list(K)] * ns, [list(faces)] * ns)


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 7), (5, 1, 1), (1, 6, 1), (3, 2, 65), (2, 70, 3)])
def test_degenerate_shapes(shape):
    rng = np.random.default_rng(sum(shape))
    faces = [(GHOST, 0.5), (MIRROR, 0), (PERIODIC, 0), (PERIODIC, 0), (HELD, 0.25), (MIRROR, 0)]
    spec = bc_spec(1, faces)
    w = W.Workload("edge", shape, spec, [rng.uniform(0, 1, shape)], 5, 0)
    ref = oracle.run(spec, w.fields, 5)[0]
    for plan in compiled_plans(w, czs=(0,)):
        got, _ = gpu_run(w, 5, plan=plan)
        assert np.max(np.abs(got[0] - ref)) <= 1e-6, plan


def test_held_and_ghost_faces_every_axis():
    shape = (9, 13, 70)
    rng = np.random.default_rng(2)
    faces = [(HELD, 1.0), (GHOST, -0.5), (HELD, 0.25), (MIRROR, 0), (GHOST, 2.0), (HELD, -1.0)]
    spec = bc_spec(2, faces)
    w = W.Workload("faces", shape, spec, [rng.uniform(0, 1, shape) for _ in range(2)], 20, 0)
    check_parity(w, 20, label="held/ghost faces")
    base = None
    for plan in compiled_plans(w, czs=(0, 3)):
        got, _ = gpu_run(w, 6, plan=plan)
        if base is None:
            base = got
        assert all(np.array_equal(a, b) for a, b in zip(got, base)), plan


@pytest.mark.parametrize("case", ["bruss256", "poll128", "front128", "faces128", "diff512", "poll512",
                                  "faces256", "held256", "bruss256ragged"])
def test_whole_tile_rows_every_plan(case):
    """Rows a whole number of x tiles long take the kernels' fast x-ghost
    path (whole periodic rows, split rows, mirror / fixed faces, fixed and
    held z planes); every plan agrees bit for bit and with the oracle."""
    if case == "bruss256":
        w = W.make_workload("brusselator256", shape=(9, 10, 256))
    elif case == "poll128":
        w = W.make_workload("pollutant512", shape=(10, 11, 128))
    elif case == "front128":
        w = W.make_workload("front384", shape=(12, 10, 128))
    elif case == "diff512":
        w = W.make_workload("diffusion512", shape=(7, 13, 512))
    elif case == "poll512":
        w = W.make_workload("pollutant512", shape=(9, 11, 512))
    elif case == "bruss256ragged":
        w = W.make_workload("brusselator256", shape=(5, 19, 256))
    elif case == "held256":
        shape = (9, 13, 256)
        rng = np.random.default_rng(3)
        faces = [(HELD, 1.0), (GHOST, -0.5), (HELD, 0.25), (MIRROR, 0), (GHOST, 2.0), (HELD, -1.0)]
        spec = bc_spec(2, faces)
        w = W.Workload("held256", shape, spec, [rng.uniform(0, 1, shape) for _ in range(2)], 6, 0)
    elif case == "faces256":
        shape = (10, 12, 256)
        rng = np.random.default_rng(9)
        faces = [(GHOST, 0.5), (MIRROR, 0), (PERIODIC, 0), (PERIODIC, 0), (HELD, 0.25), (GHOST, -1.0)]
        spec = bc_spec(1, faces)
        w = W.Workload("faces256", shape, spec, [rng.uniform(0, 1, shape)], 6, 0)
    else:
        shape = (10, 12, 128)
        rng = np.random.default_rng(9)
        faces = [(GHOST, 0.5), (MIRROR, 0), (PERIODIC, 0), (PERIODIC, 0), (HELD, 0.25), (GHOST, -1.0)]
        spec = bc_spec(2, faces)
        w = W.Workload("faces128", shape, spec, [rng.uniform(0, 1, shape) for _ in range(2)], 6, 0)
    steps = 6
    ref = oracle.run(w.spec, w.fields, steps)
    base = None
    plans = compiled_plans(w, czs=(0, 4, 7))
    if w.shape[2] in (256, 512) and w.spec.model in ("diffusion", "brusselator", "pollutant"):
        assert any(p["kernel"] == "lds" for p in plans), case
    if w.shape[2] in (256, 512) and w.spec.model in ("diffusion", "brusselator"):
        assert any(p["kernel"] == "lds2" for p in plans), case
    for plan in plans:
        got, _ = gpu_run(w, steps, plan=plan)
        if base is None:
            base = got
            for s in range(w.spec.ns):
                assert rel_l2(got[s], ref[s]) <= TOL, (case, s)
            continue
        for s in range(w.spec.ns):
            assert np.array_equal(got[s], base[s]), (case, plan, s)


@pytest.mark.parametrize("nx", [130, 200, 256, 384])
@pytest.mark.parametrize("xface", ["mirror", "periodic", "ghost", "held"])
def test_tiled_ring_x_faces(nx, xface):
    """The tiled LDS ring's 128-cell x tiles: rows that end inside a tile or
    on a tile boundary, under every x face rule (the halo units loaded for a
    periodic axis, the face rules applied at the first and last tile), for a
    one-field and a two-field model: bitwise the direct kernel's values."""
    shape = (7, 9, nx)
    rng = np.random.default_rng(nx)
    kind = {"mirror": (MIRROR, 0), "periodic": (PERIODIC, 0), "ghost": (GHOST, 0.75), "held": (HELD, 0.5)}[xface]
    faces = [kind, kind, (MIRROR, 0), (GHOST, -0.25), (HELD, 1.0), (MIRROR, 0)]
    for ns in (1, 2):
        spec = bc_spec(ns, faces)
        w = W.Workload("xfaces", shape, spec, [rng.uniform(0, 1, shape) for _ in range(ns)], 5, 0)
        plans = [p for p in compiled_plans(w, czs=(0, 3)) if p["kernel"] == "tring"]
        assert plans, (nx, xface, ns)
        base, _ = gpu_run(w, 5, plan=dict(kernel="direct"))
        for plan in plans:
            got, _ = gpu_run(w, 5, plan=plan)
            for s in range(ns):
                assert np.array_equal(got[s], base[s]), (nx, xface, ns, plan, s)


# ------------------------------------------------------ 19-point Laplacian

def as19(w, dt=None):
    """The same workload on the 19-point Laplacian of Eqs. (3)-(4): each
    species keeps its x coefficient on every axis."""
    spec = w.spec.copy()
    spec.stencil = 19
    spec.K = [[k[0]] * 3 for k in spec.K]
    if dt is not None:
        spec.dt = dt
    return W.Workload(w.name + "_19", w.shape, spec, w.fields, w.steps, w.seed)


def case19(case):
    if case == "faces70":
        shape = (9, 10, 70)
        rng = np.random.default_rng(21)
        faces = [(HELD, 1.0), (GHOST, -0.5), (PERIODIC, 0), (PERIODIC, 0), (GHOST, 2.0), (HELD, -1.0)]
        return as19(W.Workload("faces70", shape, bc_spec(2, faces, K=(0.5, 0.5, 0.5)),
                               [rng.uniform(0, 1, shape) for _ in range(2)], 6, 0))
    if case == "faces256":
        shape = (10, 12, 256)
        rng = np.random.default_rng(22)
        faces = [(GHOST, 0.5), (MIRROR, 0), (PERIODIC, 0), (PERIODIC, 0), (HELD, 0.25), (GHOST, -1.0)]
        return as19(W.Workload("faces256", shape, bc_spec(1, faces, K=(1.0, 1.0, 1.0)),
                               [rng.uniform(0, 1, shape)], 6, 0))
    if case == "ghosts256":
        # fixed ghosts of different values on x-, y+ and z-, none held: the
        # edge ghosts between two of them take the first axis's value
        shape = (8, 11, 256)
        rng = np.random.default_rng(25)
        faces = [(GHOST, 0.25), (MIRROR, 0), (MIRROR, 0), (GHOST, 0.5), (GHOST, -1.0), (MIRROR, 0)]
        return as19(W.Workload("ghosts256", shape, bc_spec(1, faces, K=(1.0, 1.0, 1.0)),
                               [rng.uniform(0, 1, shape)], 6, 0))
    if case == "held512":
        shape = (7, 9, 512)
        rng = np.random.default_rng(23)
        faces = [(HELD, 1.0), (GHOST, -0.5), (HELD, 0.25), (MIRROR, 0), (GHOST, 2.0), (HELD, -1.0)]
        return as19(W.Workload("held512", shape, bc_spec(2, faces, K=(1.0, 1.0, 1.0)),
                               [rng.uniform(0, 1, shape) for _ in range(2)], 6, 0))
    if case == "bruss256":
        return as19(W.make_workload("brusselator256", shape=(8, 10, 256)))
    if case == "bruss256ragged":
        return as19(W.make_workload("brusselator256", shape=(5, 19, 256)))
    if case == "poll256":
        return as19(W.make_workload("pollutant512", shape=(9, 11, 256)))
    if case == "front512":
        w = W.make_workload("front384", shape=(9, 10, 512))
        spec = w.spec
        spec.bc[2] = [(HELD, 0.3), (GHOST, 0.1), (GHOST, -0.2), (HELD, 0.4), (HELD, 0.5), (GHOST, 0.0)]
        spec.bc[1] = [(GHOST, 0.2), (HELD, 0.6), (MIRROR, 0), (GHOST, 0.3), (MIRROR, 0), (HELD, 0.1)]
        rng = np.random.default_rng(24)
        fields = [f.astype(np.float32).astype(np.float64) for f in w.fields]
        fields[2] = rng.uniform(-1.0, 1.0, w.shape).astype(np.float32).astype(np.float64)
        return as19(W.Workload("front512", w.shape, spec, fields, 6, 0))
    raise KeyError(case)


@pytest.mark.parametrize("case", ["faces70", "faces256", "ghosts256", "held512", "bruss256", "bruss256ragged",
                                  "poll256", "front512"])
def test_stencil19_every_plan(case):
    """The 19-point Laplacian with edge ghosts on every face kind: the
    direct and LDS-ring plans agree bit for bit and with the oracle; the
    plans that only know the 7-point form are refused."""
    w = case19(case)
    steps = 6
    ref = oracle.run(w.spec, w.fields, steps)
    plans = compiled_plans(w, czs=(0, 4, 7))
    assert all(p["kernel"] in ("direct", "lds") for p in plans), case
    if w.shape[2] in (256, 512) and w.spec.model in ("diffusion", "brusselator", "pollutant"):
        assert any(p["kernel"] == "lds" for p in plans), case
    base = None
    for plan in plans:
        got, _ = gpu_run(w, steps, plan=plan)
        if base is None:
            base = got
            for s in range(w.spec.ns):
                e = rel_l2(got[s], ref[s])
                print("%s species %d rel-L2 %.3e" % (case, s, e))
                assert e <= TOL, (case, s, e)
            continue
        for s in range(w.spec.ns):
            assert np.array_equal(got[s], base[s]), (case, plan, s)
    # the 7-point change over these steps is measurably different, so the
    # stencil took effect
    w7 = W.Workload(w.name, w.shape, w.spec.copy(), w.fields, steps, 0)
    w7.spec.stencil = 7
    got7, _ = gpu_run(w7, steps, plan=dict(kernel="direct"))
    assert any(rel_l2(got7[s] - w.fields[s], ref[s] - w.fields[s]) > 1e-3 for s in range(w.spec.ns)), case


def test_stencil19_front_chemical_potential():
    """The Cahn-Hilliard potential with the 19-point Laplacian (first pass)."""
    w = case19("front512")
    mu_ref = oracle.chemical_potential(w.spec, w.fields)
    for plan in compiled_plans(w, czs=(0,)):
        g = rd.Grid(w.shape, 3, 1.0)
        g.set_model(w.spec)
        g.set_plan(**plan)
        for s in range(3):
            g.write(s, w.fields[s])
        mu = g.chemical_potential().astype(np.float64)
        g.close()
        assert np.max(np.abs(mu - mu_ref)) <= 1e-5 * max(1.0, np.max(np.abs(mu_ref))), plan


def test_stencil19_long_run_and_graphs():
    """200 steps of 19-point diffusion on 64^3 no-flux, eager and through
    graph chunks: the oracle's answer, and mass kept to FP32 rounding."""
    import torch
    w = as19(W.make_workload("diffusion64"))
    ref = oracle.run(w.spec, w.fields, 200)
    eager = None
    for chunk in (0, 16):
        g = rd.Grid(w.shape, 1, w.spec.h, "f32", stream=torch.cuda.Stream() if chunk else None)
        g.set_model(w.spec)
        g.set_plan(graph_chunk=chunk)
        g.write(0, w.fields[0])
        g.step(120)
        g.step(80)
        got = g.read_all()
        g.close()
        if eager is None:
            eager = got
            assert rel_l2(got[0], ref[0]) <= TOL
            assert abs(got[0].sum() - w.fields[0].sum()) <= 1e-5 * w.fields[0].sum()
        assert np.array_equal(got[0], eager[0]), chunk


@pytest.mark.parametrize("name,steps", [("diffusion512", 2), ("brusselator256", 4)])
def test_stencil19_full_size_autotuned(name, steps):
    """Full-size grids on the 19-point form in the autotuned plan."""
    w = as19(W.make_workload(name))
    g = rd.Grid.from_workload(w)
    g.autotune(3)
    plan = g.plan()
    assert plan["kernel"] in (rd.KERNEL["direct"], rd.KERNEL["lds"]), plan
    g.step(steps)
    got = g.read_all()
    g.close()
    ref = oracle.run(w.spec, w.fields, steps)
    for s in range(w.spec.ns):
        e = rel_l2(got[s], ref[s])
        print("%s 19-point species %d rel-L2 %.3e plan %s" % (name, s, e, plan))
        assert e <= TOL


@pytest.mark.parametrize("case", ["diff192", "bruss196_periodic", "poll384", "faces260_held", "diff452",
                                  "diff192_19", "bruss384_19_periodic", "faces196_19_held"])
def test_partial_ring_rows_every_plan(case):
    """Rows that end inside a 256-cell chunk of the LDS ring: the lanes past
    the row end load and store nothing and the row's last cell takes its x
    face rule (a periodic wrap comes from the row's other end).  Every plan
    agrees bit for bit and with the oracle."""
    rng = np.random.default_rng(sum(map(ord, case)))
    if case.startswith("diff"):
        nx = int(case[4:7])
        shape = (7, 9, nx)
        spec = bc_spec(1, [(MIRROR, 0)] * 6, K=(1.0, 1.0, 1.0), dt=0.1)
        fields = [rng.uniform(0, 1, shape)]
    elif case.startswith("bruss"):
        nx = int(case[5:8])
        w = W.make_workload("brusselator256", shape=(6, 10, nx))
        spec, fields, shape = w.spec, w.fields, w.shape
    elif case.startswith("poll"):
        w = W.make_workload("pollutant512", shape=(8, 10, 384))
        spec, shape = w.spec, w.shape
        fields = [rng.uniform(0, 1, shape) for _ in range(spec.ns)]
    else:
        nx = int(case[5:8])
        shape = (8, 9, nx)
        faces = [(HELD, 1.0), (GHOST, -0.5), (PERIODIC, 0), (PERIODIC, 0), (GHOST, 2.0), (HELD, -1.0)]
        spec = bc_spec(2, faces, K=(1.0, 1.0, 1.0), dt=0.1)
        fields = [rng.uniform(0, 1, shape) for _ in range(2)]
    if "_19" in case:
        spec = spec.copy()
        spec.stencil = 19
        spec.K = [[k[0]] * 3 for k in spec.K]
    w = W.Workload(case, shape, spec, fields, 6, 0)
    steps = 6
    ref = oracle.run(w.spec, w.fields, steps)
    plans = compiled_plans(w, czs=(0, 4))
    assert any(p["kernel"] == "lds" for p in plans), case
    base = None
    for plan in plans:
        got, _ = gpu_run(w, steps, plan=plan)
        if base is None:
            base = got
            for s in range(w.spec.ns):
                assert rel_l2(got[s], ref[s]) <= TOL, (case, s)
            continue
        for s in range(w.spec.ns):
            assert np.array_equal(got[s], base[s]), (case, plan, s)


@pytest.mark.parametrize("case", ["bruss256", "diff512", "poll512", "faces200_held", "diff192_19", "bruss384_19"])
def test_bf16_ring_every_plan(case):
    """BF16 storage on the LDS ring (2-byte cells, 8 per 16-byte load, rows
    that end inside a load): every plan gives the same bits, and a single
    step is within one BF16 unit of the oracle's step rounded to BF16."""
    rng = np.random.default_rng(sum(map(ord, case)))
    if case == "bruss256":
        w = W.make_workload("brusselator256", shape=(6, 10, 256))
    elif case == "diff512":
        w = W.make_workload("diffusion512", shape=(7, 9, 512))
    elif case == "poll512":
        w = W.make_workload("pollutant512", shape=(8, 9, 512))
        w.fields = [rng.uniform(0, 1, w.shape) for _ in range(4)]
    elif case == "faces200_held":
        shape = (8, 9, 200)
        faces = [(HELD, 1.0), (GHOST, -0.5), (PERIODIC, 0), (PERIODIC, 0), (GHOST, 2.0), (HELD, -1.0)]
        w = W.Workload(case, shape, bc_spec(2, faces, K=(1.0, 1.0, 1.0), dt=0.1),
                       [rng.uniform(0, 1, shape) for _ in range(2)], 6, 0)
    elif case == "diff192_19":
        shape = (7, 9, 192)
        spec = bc_spec(1, [(MIRROR, 0)] * 6, K=(1.0, 1.0, 1.0), dt=0.1)
        spec.stencil = 19
        w = W.Workload(case, shape, spec, [rng.uniform(0, 1, shape)], 6, 0)
    else:
        w = W.make_workload("brusselator256", shape=(6, 8, 384))
        w.spec.stencil = 19
    fields = [round_bf16(f) for f in w.fields]
    w = W.Workload(w.name, w.shape, w.spec, fields, 6, 0)
    plans = compiled_plans(w, storage="bf16", czs=(0, 4))
    assert any(p["kernel"] == "lds" for p in plans), case
    base = None
    for plan in plans:
        got, _ = gpu_run(w, 3, storage="bf16", plan=plan)
        if base is None:
            base = got
            continue
        for s in range(w.spec.ns):
            assert np.array_equal(got[s], base[s]), (case, plan, s)
    ring = next(p for p in plans if p["kernel"] == "lds")
    one, _ = gpu_run(w, 1, storage="bf16", plan=ring)
    ref = oracle.run(w.spec, w.fields, 1)
    for s in range(w.spec.ns):
        assert np.all(np.abs(one[s] - round_bf16(ref[s])) <= ulp(ref[s], "bf16") * 1.01 + 1e-30), (case, s)


@pytest.mark.parametrize("name,shape", [("brusselator256", (6, 12, 256)), ("diffusion512", (9, 7, 512))])
def test_two_step_plans_with_graphs_and_odd_counts(name, shape):
    """Two steps per launch: graph chunks of 2, 4 and 6 steps and odd step
    counts (the last step then runs on the direct kernel) give the bits of
    single steps."""
    w = W.make_workload(name, shape=shape)
    ref, _ = gpu_run(w, 9, plan=dict(kernel="direct"))
    for vx, by, wc, d in LDS2_SHAPES:
        for chunk in (0, 2, 4, 6):
            plan = dict(kernel="lds2", vx=vx, ry=by, waves=wc, prefetch=d, cz=0, graph_chunk=chunk)
            g = rd.Grid(w.shape, w.spec.ns, w.spec.h)
            g.set_model(w.spec)
            try:
                g.set_plan(**plan)
            except rd.RDError:
                g.close()
                continue
            for s_, f in enumerate(w.fields):
                g.write(s_, f)
            g.step(3)
            g.step(6)          # 9 steps in two calls: odd, then even
            got = g.read_all()
            g.close()
            for s_ in range(w.spec.ns):
                assert np.array_equal(got[s_], ref[s_]), (plan, s_)


def test_zero_steps_is_identity():
    w = W.make_workload("pollutant512", shape=(5, 6, 7))
    got, _ = gpu_run(w, 0)
    for s in range(4):
        assert np.array_equal(got[s], w.fields[s].astype(np.float32).astype(np.float64))


# ---------------------------------------------------------------- batch

def test_batched_results_equal_alone():
    """Grids of different sizes and models stepped together in one persistent
    launch per step give bit-identical fields to each grid stepped alone."""
    import torch
    stream = torch.cuda.Stream()
    reqs = [W.Request(0, 0, 32, "diffusion", 37, 11), W.Request(1, 0, 48, "brusselator", 20, 12),
            W.Request(2, 0, 64, "diffusion", 25, 13), W.Request(3, 0, 40, "brusselator", 31, 14)]
    ws = [W.request_workload(r) for r in reqs]
    b = rd.Batch(8, 1 << 34, "f32", stream=stream)
    grids = []
    for r, w in zip(reqs, ws):
        g = rd.Grid.from_workload(w, stream=stream)
        b.add(g, r.steps)
        grids.append(g)
    finished = []
    while len(finished) < len(grids):
        finished += b.step(8)
    for r, w, g in zip(reqs, ws, grids):
        alone, _ = gpu_run(w, r.steps)
        got = g.read_all()
        for s in range(w.spec.ns):
            assert np.array_equal(got[s], alone[s]), (r, s)
        g.close()
    b.close()


def test_batched_many_items_equal_alone():
    """More work items than the persistent launch has workgroups (128^3 grids
    of 64 tiles each, mixed with small ones), so workgroups claim several
    items per step and the claim counters are reused across launches and
    ticks: every grid still matches the same grid stepped alone."""
    import torch
    stream = torch.cuda.Stream()
    reqs = [W.Request(i, 0, e, m, st, 100 + i) for i, (e, m, st) in enumerate(
        [(128, "brusselator", 9), (128, "diffusion", 6), (128, "brusselator", 7), (128, "diffusion", 9),
         (128, "brusselator", 5), (128, "diffusion", 8), (96, "brusselator", 9), (96, "diffusion", 4),
         (96, "brusselator", 6), (32, "diffusion", 9), (32, "brusselator", 3), (48, "diffusion", 7),
         (64, "brusselator", 8)])]
    ws = [W.request_workload(r) for r in reqs]
    b = rd.Batch(16, 1 << 34, "f32", stream=stream)
    grids = []
    for r, w in zip(reqs, ws):
        g = rd.Grid.from_workload(w, stream=stream)
        b.add(g, r.steps)
        grids.append(g)
    finished = []
    while len(finished) < len(grids):
        finished += b.step(4)
    for r, w, g in zip(reqs, ws, grids):
        alone, _ = gpu_run(w, r.steps)
        got = g.read_all()
        for s in range(w.spec.ns):
            assert np.array_equal(got[s], alone[s]), (r, s)
        g.close()
    b.close()


def test_batch_narrow_rows_packed_two_per_wave():
    """Rows of at most 64 cells, which the batched kernel computes two rows
    per wave (one per half wave), on uneven shapes and both face kinds
    (mirror for diffusion, periodic for the Brusselator), and a 66-cell row
    that takes the unpacked form: each matches the grid stepped alone."""
    import torch
    stream = torch.cuda.Stream()
    cases = [("diffusion64", (5, 17, 64), 7), ("brusselator256", (9, 3, 50), 5), ("brusselator256", (7, 33, 62), 6),
             ("diffusion64", (6, 20, 2), 4), ("brusselator256", (4, 18, 64), 3), ("diffusion64", (5, 9, 66), 5)]
    b = rd.Batch(len(cases), 1 << 34, "f32", stream=stream)
    grids = []
    for name, shape, steps in cases:
        w = W.make_workload(name, shape=shape)
        g = rd.Grid.from_workload(w, stream=stream)
        b.add(g, steps)
        grids.append((w, steps, g))
    finished = []
    while len(finished) < len(grids):
        finished += b.step(4)
    for w, steps, g in grids:
        alone, _ = gpu_run(w, steps)
        got = g.read_all()
        for s in range(w.spec.ns):
            assert np.array_equal(got[s], alone[s]), (w.shape, s)
        g.close()
    b.close()


def test_batch_of_more_grids_than_the_lds_lookup_holds():
    """1100 small grids (more than the batched kernel's LDS copy of the
    grids' first items holds, so items find their grid in device memory):
    every grid matches the same grid stepped alone."""
    import torch
    stream = torch.cuda.Stream()
    n = 1100
    b = rd.Batch(n, 1 << 34, "f32", stream=stream)
    grids, ws = [], []
    for i in range(n):
        r = W.Request(i, 0, 8 if i % 3 else 12, "brusselator" if i % 2 else "diffusion", 3 + i % 4, 1000 + i)
        w = W.request_workload(r)
        g = rd.Grid.from_workload(w, stream=stream)
        b.add(g, r.steps)
        grids.append((r, w, g))
    finished = []
    while len(finished) < n:
        finished += b.step(2)
    for r, w, g in grids[::97] + grids[-3:]:
        alone, _ = gpu_run(w, r.steps)
        got = g.read_all()
        for s in range(w.spec.ns):
            assert np.array_equal(got[s], alone[s]), (r, s)
    for _, _, g in grids:
        g.close()
    b.close()


def test_enqueued_device_write_equals_synchronous_write():
    """A device field written with the enqueue-only copy on the grid's own
    stream, behind steps still queued there, gives the same state as the
    synchronous copy."""
    import torch
    w = W.make_workload("brusselator256", shape=(20, 24, 72))
    stream = torch.cuda.Stream()
    outs = []
    for enqueue in (False, True):
        g = rd.Grid.from_workload(w, stream=stream)
        g.step(3)                                   # work queued on the stream
        with torch.cuda.stream(stream):
            fields = [torch.tensor(f, dtype=torch.float32, device="cuda").flip(0).contiguous()
                      for f in w.fields]
            for s, f in enumerate(fields):
                g.write(s, f, enqueue_only=enqueue)
        g.step(2)
        outs.append(g.read_all())
        g.close()
    for s in range(2):
        assert np.array_equal(outs[0][s], outs[1][s])
    with pytest.raises(rd.RDError) as ei:
        g = rd.Grid.from_workload(w)
        try:
            rd._check(rd.lib().rd_write_field(g._p, 0, rd.C.c_void_p(fields[0].data_ptr()), rd.F32, 3))
        finally:
            g.close()
    assert ei.value.code == rd.EINVAL


def test_batch_budget_and_validation():
    import torch
    stream = torch.cuda.Stream()
    w = W.request_workload(W.Request(0, 0, 32, "diffusion", 10, 1))
    need = rd.grid_bytes(w.shape, 1)
    b = rd.Batch(2, need + 10, "f32", stream=stream)
    g1 = rd.Grid.from_workload(w, stream=stream)
    g2 = rd.Grid.from_workload(w, stream=stream)
    b.add(g1, 5)
    with pytest.raises(rd.RDError) as ei:
        b.add(g2, 5)
    assert ei.value.code == rd.ENOMEM
    with pytest.raises(rd.RDError) as ei:
        g1.step(1)                       # a member is stepped by its batch only
    assert ei.value.code == rd.ESTATE
    b.remove(g1)
    b.add(g2, 5)
    b.close()
    g1.close()
    g2.close()


# ------------------------------------------------ full sizes, bench plans

@pytest.mark.parametrize("name,steps", [("front384", 3), ("pollutant512", 4), ("diffusion512", 4)])
def test_full_size_autotuned_plan_parity(name, steps):
    """The full configured grid in the autotuned plan the benchmark uses,
    against the whole-grid FP64 oracle for a few steps."""
    w = W.make_workload(name)
    g = rd.Grid.from_workload(w)
    g.autotune(2)
    g.step(steps)
    plan = g.plan()
    got = g.read_all()
    g.close()
    ref = oracle.run(w.spec, w.fields, steps)
    for s in range(w.spec.ns):
        e = rel_l2(got[s], ref[s])
        print("%s full size %d steps species %d: rel-L2 %.3e plan %s" % (name, steps, s, e, plan))
        assert e <= TOL
        ref[s] = None


def test_front_full_size_long_run_invariants():
    """front384 at full size for 400 steps: fields stay finite and sum(B+C)
    drifts only by FP32 rounding."""
    w = W.make_workload("front384")
    g = rd.Grid.from_workload(w)
    g.autotune(2)
    m0 = g.reduce(1)[0] + g.reduce(2)[0]
    g.step(400)
    m1 = g.reduce(1)[0] + g.reduce(2)[0]
    for s in range(3):
        g.reduce(s)                       # raises on NaN / Inf
    g.close()
    drift = abs(m1 - m0) / abs(m0)
    print("front384 full size, 400 steps: sum(B+C) relative drift %.3e" % drift)
    assert drift < 1e-5


def test_pollutant_full_size_mass_budget():
    """pollutant512 at full size, one step in the autotuned plan: the change of
    each species' total obeys the exact discrete budget (sources, decay,
    outflow through x+, diffusive loss at the clean-inflow face, A->B)."""
    w = W.make_workload("pollutant512")
    rng = np.random.default_rng(21)
    fields = [rng.uniform(0, 1, w.shape).astype(np.float32).astype(np.float64) for _ in range(4)]
    g = rd.Grid(w.shape, 4, 1.0)
    g.set_model(w.spec)
    g.autotune(2)
    for s in range(4):
        g.write(s, fields[s])
    before = [g.reduce(s)[0] for s in range(4)]
    g.step(1)
    after = [g.reduce(s)[0] for s in range(4)]
    g.close()
    spec = w.spec
    dt, lam, kab = spec.dt, spec.params["decay"], spec.params["kab"]
    u = spec.wind[:, None]
    for s in range(4):
        c = fields[s]
        flux = np.sum(-u * c[:, :, -1]) - spec.K[s][0] * np.sum(c[:, :, 0])
        e = sum(r for cell, sp, r in zip(*spec.sources) if sp == s)
        change = flux - lam * np.sum(c) + e
        if s == 0:
            change -= kab * np.sum(fields[0])
        if s == 1:
            change += kab * np.sum(fields[0])
        got = after[s] - before[s]
        # FP32 rounding of 33.5 M updates of size ~1: allow 1e-6 of the total
        assert abs(got - dt * change) <= 1e-6 * before[s], (s, got, dt * change)
