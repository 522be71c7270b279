"""FP64 CPU oracle for the explicit reaction-diffusion step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import this module.  It shares no code
with the HIP path: it reads a problem description made of plain numbers
(a ``workloads.ModelSpec``-like object) and numpy float64 arrays.

The arithmetic lives in ``rd_oracle.c`` (section 2, Eqs. (2) and (5), the
7-point Laplacian or the 19-point one of Eqs. (3)-(4), the boundary handling
of section 4.1, the four Table 1 model families and the pollutant model with a
height-dependent wind); see its header for the exact definition.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")

MIRROR, PERIODIC, GHOST, HELD = 0, 1, 2, 3
_KIND = {"mirror": MIRROR, "periodic": PERIODIC, "ghost": GHOST, "held": HELD}
_MODEL = {"diffusion": 0, "brusselator": 1, "front_ch": 2, "pollutant": 3, "turing": 4, "atmos": 5}
_PARAM_SLOTS = {
    "diffusion": (),
    "brusselator": ("a", "b"),
    "front_ch": ("k", "M", "kappa", "eps", "gamma", "k2"),
    "pollutant": ("decay", "kab"),
    "turing": ("alpha", "beta", "gamma"),
    "atmos": ("ux", "uy", "uz", "uz_period", "t0"),
}
_INTEGRATOR = {"euler": 1, "rk2": 2, "rk3": 3}
# constants that may be left out of a spec's params (then 0)
_OPTIONAL = ("k2", "uz_period", "t0")


class _Problem(C.Structure):
    _fields_ = [
        ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
        ("ns", C.c_int32), ("model", C.c_int32),
        ("h", C.c_double), ("dt", C.c_double),
        ("K", (C.c_double * 3) * 4),
        ("bc_kind", (C.c_int32 * 6) * 4),
        ("bc_value", (C.c_double * 6) * 4),
        ("p", C.c_double * 8),
        ("wind", C.POINTER(C.c_double)),
        ("nsrc", C.c_int64),
        ("src_cell", C.POINTER(C.c_int64)),
        ("src_species", C.POINTER(C.c_int32)),
        ("src_rate", C.POINTER(C.c_double)),
        ("stencil", C.c_int32),
        ("integrator", C.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        lib = C.CDLL(_LIBPATH)
        lib.or_run.argtypes = [C.POINTER(_Problem), C.POINTER(C.c_double), C.c_int64]
        lib.or_run.restype = C.c_int
        lib.or_mu.argtypes = [C.POINTER(_Problem), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        lib.or_mu.restype = C.c_int
        lib.or_reduce.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_double,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]
        lib.or_reduce.restype = None
        lib.or_threads.restype = C.c_int
        lib.or_set_threads.argtypes = [C.c_int]
        lib.or_set_threads.restype = C.c_int
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _problem(spec, shape):
    nz, ny, nx = shape
    P = _Problem()
    P.nx, P.ny, P.nz = nx, ny, nz
    P.ns = spec.ns
    P.model = _MODEL[spec.model]
    P.h = float(spec.h)
    P.dt = float(spec.dt)
    P.stencil = int(getattr(spec, "stencil", 7))
    P.integrator = _INTEGRATOR[getattr(spec, "integrator", "euler")]
    for s in range(spec.ns):
        for d in range(3):
            P.K[s][d] = float(spec.K[s][d])
        for f in range(6):
            kind, val = spec.bc[s][f]
            P.bc_kind[s][f] = _KIND[kind]
            P.bc_value[s][f] = float(val)
    for slot, name in enumerate(_PARAM_SLOTS[spec.model]):
        P.p[slot] = float(spec.params.get(name, 0.0) if name in _OPTIONAL else spec.params[name])
    keep = []
    if spec.model == "pollutant":
        wind = np.ascontiguousarray(spec.wind, dtype=np.float64)
        if wind.shape != (nz,):
            raise ValueError("wind must have nz entries")
        keep.append(wind)
        P.wind = _dptr(wind)
    if spec.model in ("pollutant", "atmos"):
        if spec.sources is not None and len(spec.sources[0]):
            cell = np.ascontiguousarray(spec.sources[0], dtype=np.int64)
            sp = np.ascontiguousarray(spec.sources[1], dtype=np.int32)
            rate = np.ascontiguousarray(spec.sources[2], dtype=np.float64)
            keep += [cell, sp, rate]
            P.nsrc = len(cell)
            P.src_cell = cell.ctypes.data_as(C.POINTER(C.c_int64))
            P.src_species = sp.ctypes.data_as(C.POINTER(C.c_int32))
            P.src_rate = _dptr(rate)
    return P, keep


def run(spec, fields: Sequence[np.ndarray], steps: int) -> List[np.ndarray]:
    """Advance the state ``fields`` (list of (nz,ny,nx) arrays) by ``steps``
    explicit Euler steps in FP64 and return the new fields (copies)."""
    lib = _load()
    shape = tuple(np.shape(fields[0]))
    if len(fields) != spec.ns:
        raise ValueError("need one field per species")
    state = np.ascontiguousarray(np.stack([np.asarray(f, dtype=np.float64) for f in fields]))
    P, keep = _problem(spec, shape)
    rc = lib.or_run(C.byref(P), _dptr(state), int(steps))
    if rc != 0:
        raise ValueError("oracle rejected the problem (rc=%d)" % rc)
    del keep
    return [state[s].copy() for s in range(spec.ns)]


def chemical_potential(spec, fields: Sequence[np.ndarray]) -> np.ndarray:
    """mu = gamma C^3 - eps C - kappa Lap(C) for the front model."""
    lib = _load()
    shape = tuple(np.shape(fields[0]))
    state = np.ascontiguousarray(np.stack([np.asarray(f, dtype=np.float64) for f in fields]))
    mu = np.empty(shape, dtype=np.float64)
    P, keep = _problem(spec, shape)
    if lib.or_mu(C.byref(P), _dptr(state), _dptr(mu)) != 0:
        raise ValueError("oracle rejected the problem")
    del keep
    return mu


def reduce(field: np.ndarray, h: float = 1.0):
    """(mass, energy) = (sum c h^3, sum c^2 h^3) in FP64."""
    lib = _load()
    f = np.ascontiguousarray(field, dtype=np.float64)
    nz, ny, nx = f.shape
    out = np.zeros(2)
    lib.or_reduce(nx, ny, nz, float(h), _dptr(f), _dptr(out))
    return float(out[0]), float(out[1])


def threads() -> int:
    return int(_load().or_threads())


def set_threads(n: int) -> int:
    """Run on n threads from now on; returns the number in use."""
    return int(_load().or_set_threads(int(n)))
