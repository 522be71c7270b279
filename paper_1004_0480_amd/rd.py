"""Python binding of librdmi.so (include/rd.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; this module only
converts Python/numpy/torch arguments to the C ABI and back.  There is no
fallback: if the built library is missing, importing the binding fails.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librdmi.so")

MAX_SPECIES = 4
OK, EINVAL, ENOMEM, EUNSTABLE, ESTATE, EDEVICE, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
F32, BF16, F16, F64 = 0, 1, 2, 3
STORAGE = {"f32": F32, "bf16": BF16, "f16": F16}
MODEL = {"diffusion": 0, "brusselator": 1, "front_ch": 2, "pollutant": 3, "turing": 4, "atmos": 5}
BC = {"mirror": 0, "periodic": 1, "ghost": 2, "held": 3}
KERNEL = {"auto": 0, "direct": 1, "tiled": 2, "block": 3, "lds": 4, "lds2": 5, "fused": 6, "tring": 7}
INTEGRATOR = {"euler": 1, "rk2": 2, "rk3": 3}
PARAMS = {
    "diffusion": (),
    "brusselator": ("a", "b"),
    "front_ch": ("k", "M", "kappa", "eps", "gamma", "k2"),
    "pollutant": ("decay", "kab"),
    "turing": ("alpha", "beta", "gamma"),
    "atmos": ("ux", "uy", "uz", "uz_period", "t0"),
}
OPTIONAL_PARAMS = ("k2", "uz_period", "t0")   # 0 when a spec leaves them out


class RDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("rd error %d: %s" % (code, msg))
        self.code = code


class ModelDesc(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("nspecies", C.c_int32), ("dt", C.c_double),
        ("diff", (C.c_double * 3) * MAX_SPECIES),
        ("bc_kind", (C.c_int32 * 6) * MAX_SPECIES),
        ("bc_value", (C.c_double * 6) * MAX_SPECIES),
        ("param", C.c_double * 8),
        ("wind", C.POINTER(C.c_double)), ("nwind", C.c_int64),
        ("nsrc", C.c_int64),
        ("src_cell", C.POINTER(C.c_int64)),
        ("src_species", C.POINTER(C.c_int32)),
        ("src_rate", C.POINTER(C.c_double)),
        ("stencil", C.c_int32),
        ("integrator", C.c_int32),
    ]


class Plan(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("vx", C.c_int32), ("ry", C.c_int32),
                ("waves", C.c_int32), ("cz", C.c_int32), ("prefetch", C.c_int32),
                ("order", C.c_int32), ("graph_chunk", C.c_int32)]

    def as_dict(self) -> Dict[str, int]:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None

_SIGS = {
    "rd_create_grid": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_double, C.c_int32,
                                 C.c_void_p, C.POINTER(C.c_void_p)]),
    "rd_set_model": (C.c_int, [C.c_void_p, C.POINTER(ModelDesc)]),
    "rd_write_field": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32]),
    "rd_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "rd_read_field": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32]),
    "rd_reduce": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "rd_chemical_potential": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "rd_sync": (C.c_int, [C.c_void_p]),
    "rd_destroy_grid": (C.c_int, [C.c_void_p]),
    "rd_grid_bytes": (C.c_size_t, [C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32]),
    "rd_validate_model": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_double,
                                    C.POINTER(ModelDesc)]),
    "rd_set_plan": (C.c_int, [C.c_void_p, C.POINTER(Plan)]),
    "rd_get_plan": (C.c_int, [C.c_void_p, C.POINTER(Plan)]),
    "rd_get_passes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "rd_set_rounding": (C.c_int, [C.c_void_p, C.c_int32, C.c_uint64]),
    "rd_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Plan)]),
    "rd_batch_create": (C.c_int, [C.c_int32, C.c_size_t, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "rd_batch_add": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "rd_batch_step": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_void_p), C.POINTER(C.c_int32)]),
    "rd_batch_remove": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rd_batch_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_size_t),
                                C.POINTER(C.c_int64)]),
    "rd_batch_destroy": (C.c_int, [C.c_void_p]),
    "rd_copy_probe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "rd_last_error": (C.c_char_p, []),
    "rd_abi_version": (C.c_int, []),
    "rd_source_digest": (C.c_char_p, []),
    "rd_reduce_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_int64, C.c_double,
                                    C.c_void_p, C.c_void_p]),
}


def lib():
    """The loaded librdmi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librdmi.so is not built (run python paper_1004_0480_amd/build.py); "
                               "there is no CPU fallback for the HIP path")
        # torch ships its own HIP runtime under the same soname; load it first
        # so that this library binds to it and the process has one runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def reduce_noalloc(field_ptr: int, dtype: str, shape, h: float, out_ptr: int, stream=None):
    """Mass and energy of a dense device field into two device doubles at
    out_ptr, with no allocation (rd_reduce_noalloc); asynchronous."""
    nz, ny, nx = shape
    _check(lib().rd_reduce_noalloc(C.c_void_p(field_ptr), STORAGE[dtype], nx, ny, nz, float(h),
                                   C.c_void_p(out_ptr), _stream_handle(stream)))


def source_digest() -> str:
    """Digest of the sources the loaded library was built from."""
    return lib().rd_source_digest().decode()


def check_build_matches_sources():
    """Raise if the loaded library was built from other sources than the
    csrc/ files beside it (a stale binary would test and time old kernels)."""
    from . import build as _build
    want, got = _build.source_digest(), source_digest()
    if got != want:
        raise RuntimeError("librdmi.so was built from sources %s but csrc/ hashes to %s: rebuild "
                           "(python paper_1004_0480_amd/build.py)" % (got, want))
    return got


def exported_symbols() -> List[str]:
    return list(_SIGS)


def _check(rc: int):
    if rc != OK:
        raise RDError(rc, lib().rd_last_error().decode(errors="replace"))


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)       # torch.cuda.Stream


def model_desc(spec, shape) -> Tuple[ModelDesc, list]:
    """Marshal a ModelSpec into rd_model_desc; returns (desc, arrays to keep alive)."""
    nz, ny, nx = shape
    m = ModelDesc()
    m.model = MODEL[spec.model]
    m.nspecies = spec.ns
    m.dt = float(spec.dt)
    m.stencil = int(getattr(spec, "stencil", 7))
    m.integrator = INTEGRATOR[getattr(spec, "integrator", "euler")]
    for s in range(spec.ns):
        for d in range(3):
            m.diff[s][d] = float(spec.K[s][d])
        for f in range(6):
            kind, val = spec.bc[s][f]
            m.bc_kind[s][f] = BC[kind]
            m.bc_value[s][f] = float(val)
    for slot, name in enumerate(PARAMS[spec.model]):
        m.param[slot] = float(spec.params.get(name, 0.0) if name in OPTIONAL_PARAMS else spec.params[name])
    keep = []
    if spec.wind is not None:
        wind = np.ascontiguousarray(spec.wind, dtype=np.float64)
        keep.append(wind)
        m.wind = wind.ctypes.data_as(C.POINTER(C.c_double))
        m.nwind = len(wind)
    if spec.sources is not None and len(spec.sources[0]):
        cell = np.ascontiguousarray(spec.sources[0], dtype=np.int64)
        sp = np.ascontiguousarray(spec.sources[1], dtype=np.int32)
        rate = np.ascontiguousarray(spec.sources[2], dtype=np.float64)
        keep += [cell, sp, rate]
        m.nsrc = len(cell)
        m.src_cell = cell.ctypes.data_as(C.POINTER(C.c_int64))
        m.src_species = sp.ctypes.data_as(C.POINTER(C.c_int32))
        m.src_rate = rate.ctypes.data_as(C.POINTER(C.c_double))
    return m, keep


def validate_model(spec, shape) -> int:
    """Host-only check of a model for a grid shape; returns the rd status code."""
    m, keep = model_desc(spec, shape)
    nz, ny, nx = shape
    rc = lib().rd_validate_model(nx, ny, nz, spec.ns, float(spec.h), C.byref(m))
    del keep
    return int(rc)


def grid_bytes(shape, ns: int, storage: str = "f32", with_aux: bool = False) -> int:
    nz, ny, nx = shape
    return int(lib().rd_grid_bytes(nx, ny, nz, ns, STORAGE[storage], int(with_aux)))


def last_error() -> str:
    return lib().rd_last_error().decode(errors="replace")


class Grid:
    """One simulation grid: two device buffers per species, a model and a plan."""

    def __init__(self, shape, nspecies: int, h: float = 1.0, storage: str = "f32", stream=None):
        self.shape = tuple(int(v) for v in shape)     # (nz, ny, nx)
        self.ns = int(nspecies)
        self.h = float(h)
        self.storage = storage
        self.stream = stream
        nz, ny, nx = self.shape
        p = C.c_void_p()
        _check(lib().rd_create_grid(nx, ny, nz, self.ns, self.h, STORAGE[storage],
                                    _stream_handle(stream), C.byref(p)))
        self._p = p
        self.spec = None

    @classmethod
    def from_workload(cls, w, storage: str = "f32", stream=None, plan: Optional[dict] = None):
        g = cls(w.shape, w.spec.ns, w.spec.h, storage, stream)
        g.set_model(w.spec)
        if plan:
            g.set_plan(**plan)
        for s, f in enumerate(w.fields):
            g.write(s, f)
        return g

    @property
    def handle(self):
        return self._p

    def set_model(self, spec):
        m, keep = model_desc(spec, self.shape)
        _check(lib().rd_set_model(self._p, C.byref(m)))
        del keep
        self.spec = spec

    def write(self, species: int, src, enqueue_only: bool = False):
        """Load one species from a numpy array (f64/f32) or a CUDA torch tensor.
        enqueue_only (device tensors produced on the grid's own stream): the
        copy is only enqueued on that stream; the caller keeps the tensor
        alive until the stream has passed it (tensors allocated on that
        stream are reused by torch only in stream order)."""
        if hasattr(src, "data_ptr") and getattr(src, "is_cuda", False):
            dt = {"torch.float32": F32, "torch.float64": F64, "torch.bfloat16": BF16,
                  "torch.float16": F16}[str(src.dtype)]
            if not src.is_contiguous() or tuple(src.shape) != self.shape:
                raise ValueError("device source must be contiguous with shape (nz, ny, nx)")
            if enqueue_only:
                _check(lib().rd_write_field(self._p, species, C.c_void_p(src.data_ptr()), dt, 2))
                return
            # the library reads the tensor on the grid's stream: let the stream
            # that produced it finish first
            import torch
            torch.cuda.current_stream(src.device).synchronize()
            _check(lib().rd_write_field(self._p, species, C.c_void_p(src.data_ptr()), dt, 1))
            return
        a = np.asarray(src)
        if a.shape != self.shape:
            raise ValueError("field shape %s != grid shape %s" % (a.shape, self.shape))
        if a.dtype == np.float32:
            a = np.ascontiguousarray(a)
            dt = F32
        else:
            a = np.ascontiguousarray(a, dtype=np.float64)
            dt = F64
        _check(lib().rd_write_field(self._p, species, a.ctypes.data_as(C.c_void_p), dt, 0))

    def read(self, species: int, dtype=np.float64) -> np.ndarray:
        out = np.empty(self.shape, dtype=dtype)
        dt = F64 if out.dtype == np.float64 else F32
        if out.dtype not in (np.float64, np.float32):
            raise ValueError("read into float64 or float32")
        _check(lib().rd_read_field(self._p, species, out.ctypes.data_as(C.c_void_p), dt, 0))
        return out

    def read_device(self, species: int, dst) -> None:
        """Copy one species into a contiguous float32 CUDA tensor (nz, ny, nx)
        (synchronous: the tensor is ready for any stream on return)."""
        import torch
        if str(dst.dtype) != "torch.float32" or not dst.is_contiguous() or tuple(dst.shape) != self.shape:
            raise ValueError("destination must be a contiguous float32 tensor of shape (nz, ny, nx)")
        torch.cuda.current_stream(dst.device).synchronize()
        _check(lib().rd_read_field(self._p, species, C.c_void_p(dst.data_ptr()), F32, 1))

    def read_all(self, dtype=np.float64) -> List[np.ndarray]:
        return [self.read(s, dtype) for s in range(self.ns)]

    def step(self, n: int = 1):
        _check(lib().rd_step(self._p, int(n)))

    def sync(self):
        _check(lib().rd_sync(self._p))

    def reduce(self, species: int) -> Tuple[float, float]:
        out = (C.c_double * 2)()
        rc = lib().rd_reduce(self._p, species, out)
        if rc not in (OK, ENONFINITE):
            _check(rc)
        if rc == ENONFINITE:
            raise RDError(rc, last_error())
        return float(out[0]), float(out[1])

    def chemical_potential(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float32)
        _check(lib().rd_chemical_potential(self._p, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def set_plan(self, kernel="auto", vx=0, ry=0, waves=0, cz=0, prefetch=0, order=0, graph_chunk=0):
        p = Plan(KERNEL[kernel] if isinstance(kernel, str) else int(kernel), vx, ry, waves, cz,
                 prefetch, order, graph_chunk)
        _check(lib().rd_set_plan(self._p, C.byref(p)))

    def plan(self) -> Dict[str, int]:
        p = Plan()
        _check(lib().rd_get_plan(self._p, C.byref(p)))
        return p.as_dict()

    def passes(self) -> int:
        """Kernel launches per step."""
        n = C.c_int32()
        _check(lib().rd_get_passes(self._p, C.byref(n)))
        return n.value

    def set_rounding(self, mode: str = "nearest", seed: int = 0) -> None:
        """Rounding of BF16 stores: "nearest" (even) or "stochastic"."""
        _check(lib().rd_set_rounding(self._p, {"nearest": 0, "stochastic": 1}[mode], int(seed)))

    def autotune(self, trial_steps: int = 10) -> Dict[str, int]:
        p = Plan()
        _check(lib().rd_autotune(self._p, int(trial_steps), C.byref(p)))
        return p.as_dict()

    def close(self):
        if getattr(self, "_p", None):
            _check(lib().rd_destroy_grid(self._p))
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many grids stepped together by one persistent launch per step."""

    def __init__(self, max_grids: int, hbm_budget: int, storage: str = "f32", stream=None):
        p = C.c_void_p()
        _check(lib().rd_batch_create(int(max_grids), int(hbm_budget), STORAGE[storage],
                                     _stream_handle(stream), C.byref(p)))
        self._p = p
        self.max_grids = int(max_grids)
        self._members: Dict[int, Grid] = {}

    def add(self, grid: Grid, steps: int):
        _check(lib().rd_batch_add(self._p, grid.handle, int(steps)))
        self._members[grid.handle.value] = grid

    def step(self, chunk: int) -> List[Grid]:
        fin = (C.c_void_p * self.max_grids)()
        n = C.c_int32()
        _check(lib().rd_batch_step(self._p, int(chunk), fin, C.byref(n)))
        done = []
        for i in range(n.value):
            done.append(self._members.pop(fin[i]))
        return done

    def remove(self, grid: Grid):
        _check(lib().rd_batch_remove(self._p, grid.handle))
        self._members.pop(grid.handle.value, None)

    def info(self) -> Tuple[int, int, int]:
        n, b, s = C.c_int32(), C.c_size_t(), C.c_int64()
        _check(lib().rd_batch_info(self._p, C.byref(n), C.byref(b), C.byref(s)))
        return n.value, b.value, s.value

    def close(self):
        if getattr(self, "_p", None):
            _check(lib().rd_batch_destroy(self._p))
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy_probe(dst_ptr: int, src_ptr: int, nbytes: int, stream=None):
    _check(lib().rd_copy_probe(C.c_void_p(dst_ptr), C.c_void_p(src_ptr), int(nbytes),
                               _stream_handle(stream)))
