"""Seeded synthetic workloads: problem definitions and initial fields.

This module holds parameters and seeded random draws only.  It computes no
part of the time step itself, so that the FP64 oracle and the HIP path can be
fed the very same inputs without sharing any of the method's arithmetic.

Array convention: a field is a float64 numpy array of shape (nz, ny, nx) in C
order, so x is the contiguous index, matching the C[Depth][Height][Width]
layout of the paper's kernels (Tables 4 and 5).  A state is a list of fields,
one per species.

Problem definitions follow the paper's Table 1 families (pure diffusion,
Turing-type activator/inhibitor, front + Cahn-Hilliard phase separation,
atmospheric advection-diffusion), at the sizes and parameter values of the
four single-grid workloads used throughout this package:

* ``diffusion64``      -- 64^3, D=1, h=1, dt=0.1, no-flux, Gaussian blob + noise
* ``brusselator256``   -- 256^3, Brusselator a=4.5 b=6.75 Du=1 Dv=8, periodic
* ``front384``         -- 384x384x512 (x, y, z), A held at 1 on z=0, A+B->C,
                          Cahn-Hilliard term on C (kappa=1, M=0.1)
* ``pollutant512``     -- 512x512x128, 4 species, anisotropic diffusion,
                          upwind log-profile wind in +x, decay, A->B, sources
* ``diffusion512``     -- 512^3 single-species diffusion (bandwidth probe)

the paper's own Table 1 problem set at its 192^3 grid, 19-point Laplacian:

* ``t1_diffusion192``  -- D=1, h=1, dt=0.02, 1 inside a sphere of radius 20
* ``t1_turing192``     -- activator/inhibitor, D1=5e-5, D2=5e-3, h=6.2e-3
* ``t1_front192``      -- A+B->C with redissolution A+C, Cahn-Hilliard on C,
                          A held at 10 on the x=0 plane
* ``t1_atmos192``      -- one species, wind (5, 1, 5 sin(t/500)), D=100,
                          h=100, dt=5, one point source of rate 10

and the served-batch trace (``make_trace``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# Boundary-condition kinds (one per face per species).  Faces are ordered
# x-, x+, y-, y+, z-, z+.
MIRROR = "mirror"        # no-flux / zero-gradient / outflow: ghost = adjacent cell
PERIODIC = "periodic"    # ghost = cell at the opposite end of the axis
GHOST = "ghost"          # ghost = a fixed value (inflow of clean air: 0)
HELD = "held"            # the boundary layer itself is held at a fixed value
BC_KINDS = (MIRROR, PERIODIC, GHOST, HELD)
FACES = ("x-", "x+", "y-", "y+", "z-", "z+")

MODELS = ("diffusion", "brusselator", "front_ch", "pollutant", "turing", "atmos")


@dataclass
class ModelSpec:
    """Everything that defines one explicit step, as plain numbers.

    ``K[s][d]`` is the diffusion coefficient of species ``s`` along axis ``d``
    (x, y, z) in length^2/time; ``bc[s][f]`` is ``(kind, value)`` for face
    ``f``.  ``params`` holds the model's named reaction constants.  ``wind``
    (pollutant only) is the +x wind speed per z-layer, length nz.  ``sources``
    (pollutant only) is a tuple (cell, species, rate) of equal-length arrays,
    ``cell`` the linear index z*ny*nx + y*nx + x.  ``stencil`` is the
    Laplacian: 7 (the workloads' 7-point form) or 19 (the paper's 19-point
    form, isotropic coefficients only).  ``integrator`` is "euler" (Eq. (5)),
    "rk2" or "rk3" (strong-stability-preserving Runge-Kutta of order 2 or 3
    built from Euler steps).
    """
    model: str
    ns: int
    dt: float
    h: float
    K: List[List[float]]
    bc: List[List[Tuple[str, float]]]
    params: Dict[str, float] = field(default_factory=dict)
    wind: Optional[np.ndarray] = None
    sources: Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]] = None
    stencil: int = 7
    integrator: str = "euler"

    def copy(self) -> "ModelSpec":
        return ModelSpec(self.model, self.ns, self.dt, self.h,
                         [list(r) for r in self.K],
                         [list(r) for r in self.bc], dict(self.params),
                         None if self.wind is None else self.wind.copy(),
                         None if self.sources is None else
                         tuple(a.copy() for a in self.sources), self.stencil, self.integrator)


@dataclass
class Workload:
    name: str
    shape: Tuple[int, int, int]          # (nz, ny, nx)
    spec: ModelSpec
    fields: List[np.ndarray]             # initial state, float64 (nz, ny, nx)
    steps: int
    seed: int

    @property
    def cells(self) -> int:
        nz, ny, nx = self.shape
        return nz * ny * nx


def uniform_bc(ns: int, kind: str, value: float = 0.0):
    return [[(kind, float(value))] * 6 for _ in range(ns)]


# ---------------------------------------------------------------- generators

def gaussian_blob(shape, sigma: float, seed: int, noise: float = 1e-3):
    """Amplitude-1 Gaussian centred at the grid centre ((n-1)/2 per axis) plus
    additive uniform noise in [0, noise) drawn in C order from PCG64(seed)."""
    nz, ny, nx = shape
    z = np.arange(nz, dtype=np.float64) - (nz - 1) / 2.0
    y = np.arange(ny, dtype=np.float64) - (ny - 1) / 2.0
    x = np.arange(nx, dtype=np.float64) - (nx - 1) / 2.0
    r2 = z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2
    rng = np.random.default_rng(seed)
    return np.exp(-r2 / (2.0 * sigma * sigma)) + rng.uniform(0.0, noise, size=shape)


def diffusion_spec(D: float = 1.0, dt: float = 0.1, h: float = 1.0,
                   kind: str = MIRROR, ns: int = 1) -> ModelSpec:
    return ModelSpec("diffusion", ns, dt, h, [[D, D, D] for _ in range(ns)],
                     uniform_bc(ns, kind))


def brusselator_spec(a=4.5, b=6.75, Du=1.0, Dv=8.0, dt=0.01, h=1.0,
                     kind: str = PERIODIC) -> ModelSpec:
    return ModelSpec("brusselator", 2, dt, h, [[Du] * 3, [Dv] * 3],
                     uniform_bc(2, kind), {"a": a, "b": b})


def front_spec(k=1.0, M=0.1, kappa=1.0, eps=1.0, gamma=1.0, DA=1.0, DB=1.0,
               DC=0.0, dt=0.005, h=1.0, held_value=1.0) -> ModelSpec:
    bc = uniform_bc(3, MIRROR)
    bc[0][4] = (HELD, float(held_value))     # A held on the z=0 face
    return ModelSpec("front_ch", 3, dt, h, [[DA] * 3, [DB] * 3, [DC] * 3], bc,
                     {"k": k, "M": M, "kappa": kappa, "eps": eps, "gamma": gamma})


def log_wind(nz: int, umax: float = 5.0, levels: int = 129) -> np.ndarray:
    """u(z) = umax * ln(1 + z) / ln(levels) with z the cell index."""
    z = np.arange(nz, dtype=np.float64)
    return umax * np.log1p(z) / math.log(levels)


def cfl_dt(K: Sequence[float], umax: float, h: float, cfl: float = 0.5) -> float:
    """Largest explicit step at the given CFL number for 7-point diffusion plus
    first-order upwind advection: dt * (2*(Kx+Ky+Kz)/h^2 + umax/h) = cfl."""
    return cfl / (2.0 * sum(K) / (h * h) + umax / h)


def pollutant_sources(shape, seed: int, n: int = 64, ns: int = 4, rate: float = 10.0,
                      zmax: int = 15):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, nx, n)
    ys = rng.integers(0, ny, n)
    zs = rng.integers(0, min(zmax, nz - 1) + 1, n)
    cells = (zs * ny + ys) * nx + xs
    species = np.arange(n) % ns
    return (cells.astype(np.int64), species.astype(np.int32),
            np.full(n, rate, dtype=np.float64))


def pollutant_spec(shape, seed: int, ns: int = 4, Kxy=50.0, Kz=1.0, umax=5.0,
                   decay=1e-4, kab=1e-3, h=1.0, nsrc=64, rate=10.0,
                   dt: Optional[float] = None) -> ModelSpec:
    nz = shape[0]
    K = [[Kxy, Kxy, Kz] for _ in range(ns)]
    bc = uniform_bc(ns, MIRROR)
    for s in range(ns):
        bc[s][0] = (GHOST, 0.0)              # inflow of clean air at x=0
    if dt is None:
        dt = cfl_dt(K[0], umax, h)
    return ModelSpec("pollutant", ns, dt, h, K, bc, {"decay": decay, "kab": kab},
                     wind=log_wind(nz, umax), sources=pollutant_sources(
                         shape, seed + 1000, n=nsrc, ns=ns, rate=rate))


# ----------------------------------------------- the paper's Table 1 at 192^3

def sphere(shape, radius: float):
    """1 on cells whose centre lies within `radius` of the grid centre
    ((n-1)/2 per axis), 0 elsewhere."""
    nz, ny, nx = shape
    z = np.arange(nz, dtype=np.float64) - (nz - 1) / 2.0
    y = np.arange(ny, dtype=np.float64) - (ny - 1) / 2.0
    x = np.arange(nx, dtype=np.float64) - (nx - 1) / 2.0
    r2 = z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2
    return (r2 <= radius * radius).astype(np.float64)


def turing_spec(D1=5e-5, D2=5e-3, h=6.2e-3, dt=5e-4, alpha=0.5, beta=0.09, gamma=26.0,
                stencil: int = 19) -> ModelSpec:
    return ModelSpec("turing", 2, dt, h, [[D1] * 3, [D2] * 3], uniform_bc(2, MIRROR),
                     {"alpha": alpha, "beta": beta, "gamma": gamma}, stencil=stencil)


def paper_front_spec(k1=0.2, k2=0.005, lam=1.0, eps=1.0, gamma=1.0, sigma=1.0, D1=1.0, D2=1.0,
                     dt=0.02, h=1.0, held_value=10.0, stencil: int = 19) -> ModelSpec:
    """Table 1, third row: C has no Fickian term; A is held on the x = 0 plane."""
    bc = uniform_bc(3, MIRROR)
    bc[0][0] = (HELD, float(held_value))
    return ModelSpec("front_ch", 3, dt, h, [[D1] * 3, [D2] * 3, [0.0] * 3], bc,
                     {"k": k1, "k2": k2, "M": lam, "kappa": sigma, "eps": eps, "gamma": gamma},
                     stencil=stencil)


def atmos_spec(shape, D=100.0, h=100.0, dt=5.0, ux=5.0, uy=1.0, uz=5.0, period=500.0, rate=10.0,
               source=None, stencil: int = 19) -> ModelSpec:
    """Table 1, last row.  The source cell is not given in the paper: here it
    sits a quarter of the way along x (upwind), centred in y and z."""
    nz, ny, nx = shape
    sx, sy, sz = source if source is not None else (nx // 4, ny // 2, nz // 2)
    cells = np.array([(sz * ny + sy) * nx + sx], np.int64)
    return ModelSpec("atmos", 1, dt, h, [[D] * 3], uniform_bc(1, MIRROR),
                     {"ux": ux, "uy": uy, "uz": uz, "uz_period": period, "t0": 0.0},
                     sources=(cells, np.zeros(1, np.int32), np.array([rate])), stencil=stencil)


# ------------------------------------------------------------------ catalogue

DEFAULT_SHAPES = {
    "diffusion64": (64, 64, 64),
    "brusselator256": (256, 256, 256),
    "front384": (512, 384, 384),
    "pollutant512": (128, 512, 512),
    "diffusion512": (512, 512, 512),
    "t1_diffusion192": (192, 192, 192),
    "t1_turing192": (192, 192, 192),
    "t1_front192": (192, 192, 192),
    "t1_atmos192": (192, 192, 192),
}
DEFAULT_STEPS = {"diffusion64": 100, "brusselator256": 2000, "front384": 5000,
                 "pollutant512": 3000, "diffusion512": 100, "t1_diffusion192": 1000,
                 "t1_turing192": 1000, "t1_front192": 1000, "t1_atmos192": 1000}
DEFAULT_SEEDS = {"diffusion64": 0, "brusselator256": 1, "front384": 2,
                 "pollutant512": 3, "diffusion512": 5, "t1_diffusion192": 6,
                 "t1_turing192": 7, "t1_front192": 8, "t1_atmos192": 9}


def make_workload(name: str, shape: Optional[Tuple[int, int, int]] = None,
                  seed: Optional[int] = None, steps: Optional[int] = None) -> Workload:
    """Build a named workload, optionally at another (nz, ny, nx) shape."""
    shape = tuple(shape or DEFAULT_SHAPES[name])
    seed = DEFAULT_SEEDS[name] if seed is None else seed
    steps = DEFAULT_STEPS[name] if steps is None else steps
    nz, ny, nx = shape
    if name in ("diffusion64", "diffusion512"):
        sigma = 6.0 * max(shape) / 64.0
        spec = diffusion_spec()
        fields = [gaussian_blob(shape, sigma, seed)]
    elif name == "brusselator256":
        spec = brusselator_spec()
        a, b = spec.params["a"], spec.params["b"]
        rng = np.random.default_rng(seed)
        xi_u = rng.uniform(-0.01, 0.01, size=shape)
        xi_v = rng.uniform(-0.01, 0.01, size=shape)
        fields = [a * (1.0 + xi_u), (b / a) * (1.0 + xi_v)]
    elif name == "front384":
        spec = front_spec()
        rng = np.random.default_rng(seed)
        A = np.zeros(shape)
        A[0] = spec.bc[0][4][1]
        B = 0.1 * (1.0 + rng.uniform(-0.01, 0.01, size=shape))
        C = np.full(shape, -1.0)
        fields = [A, B, C]
    elif name == "pollutant512":
        spec = pollutant_spec(shape, seed)
        fields = [np.zeros(shape) for _ in range(spec.ns)]
    elif name == "t1_diffusion192":
        spec = ModelSpec("diffusion", 1, 0.02, 1.0, [[1.0] * 3], uniform_bc(1, MIRROR), stencil=19)
        fields = [sphere(shape, 20.0)]
    elif name == "t1_turing192":
        spec = turing_spec()
        rng = np.random.default_rng(seed)
        fields = [1.0 + rng.uniform(-5e-4, 5e-4, size=shape) for _ in range(2)]
    elif name == "t1_front192":
        spec = paper_front_spec()
        A = np.zeros(shape)
        A[:, :, 0] = spec.bc[0][0][1]
        fields = [A, np.ones(shape), np.full(shape, -1.0)]
    elif name == "t1_atmos192":
        spec = atmos_spec(shape)
        fields = [np.zeros(shape)]
    else:
        raise KeyError(name)
    return Workload(name, shape, spec, fields, steps, seed)


# --------------------------------------------------------------- served batch

SERVE_EDGES = (32, 48, 64, 96, 128)


@dataclass
class Request:
    rid: int
    gap: float          # exponential inter-arrival gap at unit rate
    edge: int
    model: str          # "diffusion" | "brusselator"
    steps: int
    seed: int


def make_trace(n: int = 4096, seed: int = 4, edges=SERVE_EDGES,
               min_steps: int = 200, max_steps: int = 2000) -> List[Request]:
    """Request trace for the served batch: unit-rate exponential gaps (scale
    by 1/lambda for arrival times), edge uniform over ``edges``, model 50/50,
    steps uniform in [min_steps, max_steps], per-request seeds spawned from
    one SeedSequence."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0, n)
    eidx = rng.integers(0, len(edges), n)
    brus = rng.random(n) < 0.5
    steps = rng.integers(min_steps, max_steps + 1, n)
    kids = np.random.SeedSequence(seed).spawn(n)
    out = []
    for i in range(n):
        out.append(Request(i, float(gaps[i]), int(edges[eidx[i]]),
                           "brusselator" if brus[i] else "diffusion",
                           int(steps[i]), int(kids[i].generate_state(1)[0])))
    return out


def request_workload(req: Request) -> Workload:
    """Initial state of one served request: the diffusion64 or brusselator256
    problem at the request's cube edge, seeded with the request's own seed."""
    shape = (req.edge,) * 3
    if req.model == "diffusion":
        w = Workload("diffusion", shape, diffusion_spec(),
                     [gaussian_blob(shape, 6.0, req.seed)], req.steps, req.seed)
        return w
    w = make_workload("brusselator256", shape=shape, seed=req.seed, steps=req.steps)
    w.name = "brusselator"
    return w


def request_fields_device(req: Request, device="cuda"):
    """Initial state of a served request generated on the device (torch,
    float32), seeded by the request: the diffusion64 or brusselator256 initial
    condition at the request's edge, with the noise drawn by a seeded device
    generator (a different but equally seeded recipe from the numpy one, used
    where host generation of thousands of grids would dominate)."""
    import torch
    n = req.edge
    gen = torch.Generator(device=device)
    gen.manual_seed(int(req.seed) & 0x7FFFFFFFFFFFFFFF)
    if req.model == "diffusion":
        c = torch.arange(n, device=device, dtype=torch.float32) - (n - 1) / 2.0
        r2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
        blob = torch.exp(-r2 / (2.0 * 6.0 * 6.0))
        return [blob + 1e-3 * torch.rand((n, n, n), generator=gen, device=device)]
    spec = brusselator_spec()
    a, b = spec.params["a"], spec.params["b"]
    xu = torch.rand((n, n, n), generator=gen, device=device) * 0.02 - 0.01
    xv = torch.rand((n, n, n), generator=gen, device=device) * 0.02 - 0.01
    return [a * (1.0 + xu), (b / a) * (1.0 + xv)]


def request_spec(req: Request) -> ModelSpec:
    return diffusion_spec() if req.model == "diffusion" else brusselator_spec()
