"""Host-side checks of the C ABI: the library loads, exports every function
include/rd.h declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1004_0480_amd import rd
from paper_1004_0480_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "rd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rd_[a-z_0-9]+)\s*\(", text)))


def test_library_loads_and_exports_header_functions():
    L = rd.lib()
    names = header_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(rd.exported_symbols())
    assert L.rd_abi_version() == 1


def test_library_built_from_these_sources():
    """The digest compiled into the library is the digest of csrc/ now."""
    from paper_1004_0480_amd import build
    assert rd.source_digest() == build.source_digest()
    assert rd.check_build_matches_sources() == build.source_digest()


def test_model_desc_layout_matches_header():
    # int32 model, int32 nspecies, double dt, 4x3 double, 4x6 int32, 4x6 double,
    # 8 double, ptr, int64, int64, ptr, ptr, ptr, int32 stencil (+4 padding)
    assert C.sizeof(rd.ModelDesc) == 4 + 4 + 8 + 96 + 96 + 192 + 64 + 8 + 8 + 8 + 8 + 8 + 8 + 8
    assert C.sizeof(rd.Plan) == 32


@pytest.mark.parametrize("args", [
    (0, 4, 4, 1, 1.0, rd.F32), (4, 0, 4, 1, 1.0, rd.F32), (4, 4, -1, 1, 1.0, rd.F32),
    (4, 4, 4, 0, 1.0, rd.F32), (4, 4, 4, 5, 1.0, rd.F32), (4, 4, 4, 1, 0.0, rd.F32),
    (4, 4, 4, 1, float("nan"), rd.F32), (4, 4, 4, 1, 1.0, rd.F64), (4, 4, 4, 1, 1.0, 7),
])
def test_create_grid_rejects_bad_arguments(args):
    p = C.c_void_p()
    assert rd.lib().rd_create_grid(*args, None, C.byref(p)) == rd.EINVAL
    assert p.value is None
    assert rd.last_error()


def test_null_handles_rejected():
    L = rd.lib()
    assert L.rd_step(None, 1) == rd.EINVAL
    assert L.rd_destroy_grid(None) == rd.EINVAL
    assert L.rd_set_model(None, None) == rd.EINVAL
    assert L.rd_batch_step(None, 1, None, None) == rd.EINVAL
    assert L.rd_copy_probe(None, None, 16, None) == rd.EINVAL
    assert L.rd_get_passes(None, None) == rd.EINVAL
    assert L.rd_create_grid(4, 4, 4, 1, 1.0, rd.F32, None, None) == rd.EINVAL


def test_validate_accepts_the_four_workloads():
    for name in ("diffusion64", "brusselator256", "front384", "pollutant512", "diffusion512"):
        w = W.make_workload(name, shape=(8, 9, 10))
        assert rd.validate_model(w.spec, w.shape) == rd.OK, (name, rd.last_error())


def test_validate_full_size_workloads():
    for name in ("brusselator256", "front384"):
        spec = W.make_workload(name, shape=(4, 4, 4)).spec
        assert rd.validate_model(spec, W.DEFAULT_SHAPES[name]) == rd.OK
    shape = W.DEFAULT_SHAPES["pollutant512"]
    spec = W.pollutant_spec(shape, 3)
    assert rd.validate_model(spec, shape) == rd.OK


def test_validate_rejects_unstable_dt():
    spec = W.diffusion_spec(dt=0.17)          # 0.17 * 6 > 1
    assert rd.validate_model(spec, (8, 8, 8)) == rd.EUNSTABLE
    assert rd.validate_model(W.diffusion_spec(dt=1 / 6), (8, 8, 8)) == rd.OK
    b = W.brusselator_spec(dt=0.03)           # Dv = 8: 0.03 * 48 > 1
    assert rd.validate_model(b, (8, 8, 8)) == rd.EUNSTABLE
    shape = (16, 8, 8)
    p = W.pollutant_spec(shape, 1, dt=0.1)    # the advective-only CFL reading
    assert rd.validate_model(p, shape) == rd.EUNSTABLE
    f = W.front_spec(M=10.0)
    assert rd.validate_model(f, (8, 8, 8)) == rd.EUNSTABLE


def test_validate_rejects_bad_models():
    shape = (6, 6, 6)
    s = W.diffusion_spec()
    s.bc[0][0] = ("periodic", 0.0)            # periodic on one face only
    assert rd.validate_model(s, shape) == rd.EINVAL
    s = W.diffusion_spec()
    s.K[0][1] = -1.0
    assert rd.validate_model(s, shape) == rd.EINVAL
    s = W.brusselator_spec()
    s.ns = 3
    s.K.append([1, 1, 1])
    s.bc.append(s.bc[0])
    assert rd.validate_model(s, shape) == rd.EINVAL
    p = W.pollutant_spec(shape, 1)
    p.wind = p.wind[:-1]                      # wrong length
    assert rd.validate_model(p, shape) == rd.EINVAL
    p = W.pollutant_spec(shape, 1)
    p.wind = -p.wind - 1.0                    # upwind needs u >= 0
    assert rd.validate_model(p, shape) == rd.EINVAL
    p = W.pollutant_spec(shape, 1)
    p.sources = (np.array([6 ** 3], np.int64), np.array([0], np.int32), np.array([1.0]))
    assert rd.validate_model(p, shape) == rd.EINVAL
    p = W.pollutant_spec(shape, 1)
    p.sources = (np.array([3], np.int64), np.array([4], np.int32), np.array([1.0]))
    assert rd.validate_model(p, shape) == rd.EINVAL
    s = W.diffusion_spec()
    s.dt = float("inf")
    assert rd.validate_model(s, shape) == rd.EINVAL


def test_validate_stencil19():
    shape = (8, 8, 8)
    s = W.diffusion_spec(dt=0.2)
    s.stencil = 19
    assert rd.validate_model(s, shape) == rd.OK           # 0.2 * 4 <= 1
    s.dt = 0.26
    assert rd.validate_model(s, shape) == rd.EUNSTABLE    # 0.26 * 4 > 1
    a = W.diffusion_spec(dt=0.05)
    a.K[0][2] = 0.5
    a.stencil = 19
    assert rd.validate_model(a, shape) == rd.EINVAL       # anisotropic
    a.stencil = 9
    assert rd.validate_model(a, shape) == rd.EINVAL
    p = W.pollutant_spec(shape, 1)
    p.stencil = 19                                        # Kx = Ky = 50, Kz = 1
    assert rd.validate_model(p, shape) == rd.EINVAL


def test_grid_bytes():
    b = rd.grid_bytes((64, 64, 64), 1, "f32")
    assert b >= 2 * 64 ** 3 * 4
    assert rd.grid_bytes((64, 64, 64), 1, "bf16") < b
    assert rd.grid_bytes((64, 64, 64), 3, "f32", with_aux=True) > 3 * b
    # rows are padded to 64 elements
    assert rd.grid_bytes((8, 8, 33), 1, "f32") == rd.grid_bytes((8, 8, 64), 1, "f32")
    assert rd.grid_bytes((0, 8, 8), 1, "f32") == 0


def test_validate_table1_workloads():
    """The paper's Table 1 problems at 192^3 (19-point) pass the checks; each
    is rejected past its own stability bound or with a bad parameter."""
    for name in ("t1_diffusion192", "t1_turing192", "t1_front192", "t1_atmos192"):
        spec = W.make_workload(name, shape=(4, 4, 4)).spec
        assert spec.stencil == 19
        assert rd.validate_model(W.make_workload(name, shape=(8, 9, 10)).spec, (8, 9, 10)) == rd.OK, name
        if name != "t1_atmos192":
            assert rd.validate_model(spec, W.DEFAULT_SHAPES[name]) == rd.OK, (name, rd.last_error())
    shape = W.DEFAULT_SHAPES["t1_atmos192"]
    a = W.atmos_spec(shape)
    assert rd.validate_model(a, shape) == rd.OK
    # 5 * (4 * 100 / 100^2 + (5 + 1 + 5) / 100) = 0.75; at dt = 7: 1.05
    a.dt = 7.0
    assert rd.validate_model(a, shape) == rd.EUNSTABLE
    a = W.atmos_spec(shape)
    a.params["uz_period"] = -1.0
    assert rd.validate_model(a, shape) == rd.EINVAL
    t = W.turing_spec()
    t.dt = 2e-3                                           # 4 D2 dt / h^2 = 1.04
    assert rd.validate_model(t, (8, 8, 8)) == rd.EUNSTABLE
    f = W.paper_front_spec()
    f.params["k2"] = -0.1
    assert rd.validate_model(f, (8, 8, 8)) == rd.EINVAL
    t = W.turing_spec()
    t.ns = 3
    t.K.append([1e-5] * 3)
    t.bc.append(t.bc[0])
    assert rd.validate_model(t, (8, 8, 8)) == rd.EINVAL
    d = W.make_workload("t1_diffusion192", shape=(8, 8, 8)).spec
    d.sources = (np.array([3], np.int64), np.array([0], np.int32), np.array([1.0]))
    assert rd.validate_model(d, (8, 8, 8)) == rd.EINVAL   # sources need a source model
