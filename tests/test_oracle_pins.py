"""Pins of the FP64 oracle against closed forms, invariants and special cases.

None of these re-type the oracle's formula: each compares the oracle's
output with something the mathematics fixes independently -- the exact
Laplacian of a quadratic, the exact per-step factor of a discrete Fourier
mode, the full separable cosine-transform solution of the diffusion problem,
conservation laws, scalar ODE recurrences of uniform fields, the exact
one-cell shift of unit-CFL upwinding, and a 1D recurrence of a held layer.
"""
import math

import numpy as np
import pytest

from paper_1004_0480_amd import workloads as W
from paper_1004_0480_amd.workloads import GHOST, HELD, MIRROR, PERIODIC, ModelSpec, uniform_bc

pytestmark = pytest.mark.filterwarnings("ignore")


def grid_idx(shape):
    nz, ny, nx = shape
    return np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")


def diff_spec(K, dt, h=1.0, bc=None, ns=1):
    return ModelSpec("diffusion", ns, dt, h, [list(K)] * ns,
                     bc if bc is not None else uniform_bc(ns, MIRROR))


def axis_bc(kinds, ns=1, value=0.0):
    """kinds = (kx, ky, kz) applied to both faces of each axis."""
    return [[(kinds[a // 2], value) for a in range(6)] for _ in range(ns)]


# ------------------------------------------------------------------ P1

@pytest.mark.parametrize("h", [1.0, 2.0])
def test_quadratic_field_exact_laplacian(oracle, h):
    """Section 2: a 7-point Laplacian is exact on quadratics, so one Euler
    step adds dt * 2 * (alpha Kx + beta Ky + gamma Kz) / h^2 exactly."""
    shape = (6, 7, 9)
    k, j, i = grid_idx(shape)
    al, be, ga = 3, -2, 5
    c0 = (al * i**2 + be * j**2 + ga * k**2 + 4 * i - 7 * j + 2 * k + 11).astype(float)
    K = [2.0, 3.0, 0.5]
    dt = 0.125
    out = oracle.run(diff_spec(K, dt, h), [c0], 1)[0]
    expect = c0 + dt * 2.0 * (al * K[0] + be * K[1] + ga * K[2]) / (h * h)
    inner = (slice(1, -1),) * 3
    assert np.array_equal(out[inner], expect[inner])


def test_chemical_potential_of_quadratic(oracle):
    """mu = gamma c^3 - eps c - kappa Lap(c), Lap exact on a quadratic."""
    shape = (5, 6, 7)
    k, j, i = grid_idx(shape)
    c = (i**2 - 2 * j**2 + 3 * k**2 + i - 3).astype(float)
    spec = W.front_spec(k=0.0, kappa=0.5, eps=3.0, gamma=2.0)
    mu = oracle.chemical_potential(spec, [np.zeros(shape), np.zeros(shape), c])
    expect = 2.0 * c**3 - 3.0 * c - 0.5 * 2.0 * (1 - 2 + 3)
    inner = (slice(1, -1),) * 3
    assert np.array_equal(mu[inner], expect[inner])


# ------------------------------------------------------------------ P2

def mode_1d(kind, n, q, h):
    """Eigenvector and eigenvalue of the 1D 3-point operator (c[-1]+c[+1]-2c)/h^2
    on n cells under the face rule ``kind`` applied at both ends."""
    i = np.arange(n, dtype=float)
    if kind == MIRROR:        # cell-centred reflection: DCT-II basis
        return np.cos(np.pi * q * (i + 0.5) / n), -4 * np.sin(np.pi * q / (2 * n)) ** 2 / h**2
    if kind == PERIODIC:      # any phase of the q-th harmonic
        return np.cos(2 * np.pi * q * i / n + 0.3), -4 * np.sin(np.pi * q / n) ** 2 / h**2
    if kind == GHOST:         # zero ghosts: discrete sine basis
        return (np.sin(np.pi * q * (i + 1) / (n + 1)),
                -4 * np.sin(np.pi * q / (2 * (n + 1))) ** 2 / h**2)
    raise ValueError(kind)


@pytest.mark.parametrize("kinds", [(MIRROR, MIRROR, MIRROR), (PERIODIC, PERIODIC, PERIODIC),
                                   (GHOST, GHOST, GHOST), (PERIODIC, MIRROR, GHOST),
                                   (GHOST, PERIODIC, MIRROR), (MIRROR, GHOST, PERIODIC)])
def test_fourier_mode_decay_factor(oracle, kinds):
    """Each separable mode is multiplied by g = 1 + dt sum_d K_d lambda_d per
    step, so after n steps its amplitude is g^n exactly (up to rounding)."""
    shape = (5, 6, 11)
    nz, ny, nx = shape
    h, K, dt, n = 1.3, [0.9, 0.4, 0.7], 0.2, 25
    vx, lx = mode_1d(kinds[0], nx, 2, h)
    vy, ly = mode_1d(kinds[1], ny, 1, h)
    vz, lz = mode_1d(kinds[2], nz, 3, h)
    mode = vz[:, None, None] * vy[None, :, None] * vx[None, None, :]
    g = 1 + dt * (K[0] * lx + K[1] * ly + K[2] * lz)
    out = oracle.run(diff_spec(K, dt, h, axis_bc(kinds)), [mode], n)[0]
    assert np.max(np.abs(out - g**n * mode)) < 1e-14


# 19-point Laplacian of Eqs. (3)-(4).  Each 1D mode above satisfies
# v(i-1) + v(i+1) = s v(i) with s = 2 + h^2 lambda, so a separable mode is an
# eigenvector of the 19-point sum: centre -24, faces 2 s_d, edges s_d s_e.
# For periodic modes s = 2 cos(theta) and the symbol is the paper's
# (4 sum cos + 4 sum cos cos - 24) / (6 h^2).

def spec19(D, dt, h, bc, ns=1):
    return ModelSpec("diffusion", ns, dt, h, [[D, D, D]] * ns, bc, stencil=19)


@pytest.mark.parametrize("kinds", [(MIRROR, MIRROR, MIRROR), (PERIODIC, PERIODIC, PERIODIC),
                                   (GHOST, GHOST, GHOST), (PERIODIC, MIRROR, GHOST),
                                   (GHOST, PERIODIC, MIRROR), (MIRROR, GHOST, PERIODIC)])
def test_fourier_mode_decay_factor_19(oracle, kinds):
    shape = (5, 6, 11)
    nz, ny, nx = shape
    h, D, dt, n = 1.3, 0.6, 0.2, 25
    vx, lx = mode_1d(kinds[0], nx, 2, h)
    vy, ly = mode_1d(kinds[1], ny, 1, h)
    vz, lz = mode_1d(kinds[2], nz, 3, h)
    sx, sy, sz = (2 + h * h * l for l in (lx, ly, lz))
    mode = vz[:, None, None] * vy[None, :, None] * vx[None, None, :]
    lam = (-24 + 2 * (sx + sy + sz) + (sx * sy + sx * sz + sy * sz)) / (6 * h * h)
    g = 1 + dt * D * lam
    out = oracle.run(spec19(D, dt, h, axis_bc(kinds)), [mode], n)[0]
    assert np.max(np.abs(out - g**n * mode)) < 1e-14


def test_periodic_symbol_19_is_the_papers():
    """The closed form used above equals the paper's cosine symbol."""
    th = np.linspace(0, np.pi, 7)
    a, b, c = np.meshgrid(th, th, th, indexing="ij")
    s = [2 * np.cos(t) for t in (a, b, c)]
    ours = -24 + 2 * sum(s) + (s[0] * s[1] + s[0] * s[2] + s[1] * s[2])
    papers = 4 * (np.cos(a) + np.cos(b) + np.cos(c)) + 4 * (
        np.cos(a) * np.cos(b) + np.cos(a) * np.cos(c) + np.cos(b) * np.cos(c)) - 24
    assert np.allclose(ours, papers, atol=1e-12)


@pytest.mark.parametrize("h", [1.0, 2.0])
def test_quadratic_field_exact_laplacian_19(oracle, h):
    """The 19-point form is exact on quadratics, cross terms included (they
    vanish), so one step adds dt * D * 2 (alpha + beta + gamma) / h^2."""
    shape = (6, 7, 9)
    k, j, i = grid_idx(shape)
    al, be, ga = 3, -2, 5
    c0 = (al * i**2 + be * j**2 + ga * k**2 + 2 * i * j - 3 * j * k + i * k
          + 4 * i - 7 * j + 2 * k + 11).astype(float)
    D, dt = 2.0, 0.125
    bc = uniform_bc(1, MIRROR)
    out = oracle.run(spec19(D, dt, h, bc), [c0], 1)[0]
    expect = c0 + dt * D * 2.0 * (al + be + ga) / (h * h)
    inner = (slice(1, -1),) * 3
    assert np.array_equal(out[inner], expect[inner])


def test_stencil19_mass_conserved(oracle):
    """No-flux (mirror, edge ghosts included) and periodic faces conserve sum(c)."""
    rng = np.random.default_rng(19)
    shape = (7, 8, 9)
    c0 = rng.uniform(0, 1, shape)
    for kind in (MIRROR, PERIODIC):
        out = oracle.run(spec19(1.0, 0.1, 1.0, uniform_bc(1, kind)), [c0], 20)[0]
        assert abs(out.sum() - c0.sum()) <= 1e-12 * c0.sum()


def test_stencil19_needs_isotropic_coefficients(oracle):
    spec = ModelSpec("diffusion", 1, 0.1, 1.0, [[1.0, 1.0, 0.5]], uniform_bc(1, MIRROR), stencil=19)
    with pytest.raises(Exception):
        oracle.run(spec, [np.zeros((3, 3, 3))], 1)


# ------------------------------------------------------------------ P3

def dct_basis(n):
    i = np.arange(n)
    V = np.cos(np.pi * np.outer(i + 0.5, np.arange(n)) / n)
    return V / np.linalg.norm(V, axis=0)


def test_diffusion64_closed_form(oracle):
    """The whole 64^3 no-flux diffusion run: the mirror-ghost operator is
    diagonal in the separable cosine basis, so c_n = V (g^n * V^T c_0)."""
    w = W.make_workload("diffusion64")
    nz, ny, nx = w.shape
    D, dt, h = w.spec.K[0][0], w.spec.dt, w.spec.h
    V = [dct_basis(n) for n in (nz, ny, nx)]
    lam = [-4 * np.sin(np.pi * np.arange(n) / (2 * n)) ** 2 / h**2 for n in (nz, ny, nx)]
    a = np.einsum("zk,yj,xi,zyx->kji", V[0], V[1], V[2], w.fields[0], optimize=True)
    g = 1 + dt * D * (lam[0][:, None, None] + lam[1][None, :, None] + lam[2][None, None, :])
    expect = np.einsum("zk,yj,xi,kji->zyx", V[0], V[1], V[2], a * g**w.steps, optimize=True)
    out = oracle.run(w.spec, w.fields, w.steps)[0]
    assert np.max(np.abs(out - expect)) < 1e-13


# ------------------------------------------------------------------ P4 / P5

@pytest.mark.parametrize("kind", [MIRROR, PERIODIC])
def test_mass_conserved_without_reaction(oracle, kind):
    shape = (7, 9, 10)
    rng = np.random.default_rng(7)
    c0 = rng.uniform(0, 1, shape)
    out = oracle.run(diff_spec([1.0, 0.5, 2.0], 0.05, bc=uniform_bc(1, kind)), [c0], 40)[0]
    m0, m1 = math.fsum(c0.ravel()), math.fsum(out.ravel())
    assert abs(m1 - m0) <= 1e-13 * abs(m0)


def test_energy_non_increasing(oracle):
    """dt = 0.1 <= h^2 / (6 D): every mode factor lies in [-1, 1]."""
    shape = (8, 8, 8)
    c = np.random.default_rng(3).uniform(-1, 1, shape)
    spec = W.diffusion_spec()
    e_prev = np.sum(c * c)
    for _ in range(15):
        c = oracle.run(spec, [c], 1)[0]
        e = np.sum(c * c)
        assert e <= e_prev * (1 + 1e-15)
        e_prev = e


def test_front_conserves_b_plus_c(oracle):
    """B and C have no-flux faces and the reaction moves one B into one C, the
    Cahn-Hilliard term is a divergence: sum(B + C) is invariant."""
    w = W.make_workload("front384", shape=(9, 6, 7))
    rng = np.random.default_rng(11)
    fields = [w.fields[0], w.fields[1], rng.uniform(-1, 1, w.shape)]
    out = oracle.run(w.spec, fields, 30)
    s0 = math.fsum((fields[1] + fields[2]).ravel())
    s1 = math.fsum((out[1] + out[2]).ravel())
    assert abs(s1 - s0) < 1e-12 * np.sum(np.abs(fields[1]) + np.abs(fields[2]))


def test_front_without_reaction_conserves_c(oracle):
    w = W.make_workload("front384", shape=(6, 7, 5))
    w.spec.params["k"] = 0.0
    rng = np.random.default_rng(12)
    C0 = rng.uniform(-1, 1, w.shape)
    out = oracle.run(w.spec, [w.fields[0], w.fields[1], C0], 25)
    assert abs(math.fsum(out[2].ravel()) - math.fsum(C0.ravel())) < 1e-12 * C0.size


def _face_axis_slices(face, n):
    """Index tuple of the cell layer at distance ``n`` from ``face`` (0..5)."""
    axis = 2 - face // 2          # arrays are [z][y][x]
    idx = [slice(None)] * 3
    idx[axis] = n if face % 2 == 0 else -1 - n
    return tuple(idx)


@pytest.mark.parametrize("face", range(6))
@pytest.mark.parametrize("h", [1.0, 2.0])
def test_mu_ghost_is_mirror_closed_form(oracle, face, h):
    """Section 4.1: the second Laplacian of the Cahn-Hilliard term runs on mu
    after the boundary rule is applied again -- the no-flux (mirror) rule on
    every face, whatever fixed ghost C has.  C uniform at c0 with one face a
    fixed ghost g: Lap(C) is (g - c0)/h^2 on that face's layer and 0 elsewhere,
    so mu drops by kappa (g - c0)/h^2 there, and with mu mirrored the step moves
    exactly dt M kappa (g - c0)/h^4 from the second layer into the first.  (With
    g as mu's ghost as well the first layer would change by a different amount.)"""
    shape = (6, 5, 7)
    c0, g, M, kappa, dt = 0.5, -0.75, 0.1, 1.5, 1.0 / 512
    spec = W.front_spec(k=0.0, M=M, kappa=kappa, eps=1.0, gamma=1.0, DA=0.0, DB=0.0, DC=0.0, dt=dt, h=h)
    spec.bc[0][4] = (MIRROR, 0.0)
    spec.bc[2][face] = (GHOST, g)
    zero = np.zeros(shape)
    out = oracle.run(spec, [zero, zero, np.full(shape, c0)], 1)[2]
    d = dt * M * kappa * (g - c0) / h**4
    expect = np.full(shape, c0)
    expect[_face_axis_slices(face, 0)] += d
    expect[_face_axis_slices(face, 1)] -= d
    assert np.allclose(out, expect, rtol=0, atol=1e-15)
    assert abs(out[_face_axis_slices(face, 0)][0, 0] - (c0 + d)) < 1e-15


@pytest.mark.parametrize("stencil", [7, 19])
def test_mu_mirror_conserves_c_with_fixed_and_periodic_faces(oracle, stencil):
    """With A = B = 0 and no Fickian term, C changes by M Lap(mu) only.  mu's
    mirror ghosts make that a sum of fluxes that cancel, so sum(C) is
    invariant even where C itself has fixed ghost values or a periodic axis
    (mu taking C's fixed values as ghosts would add a boundary flux)."""
    shape = (7, 6, 5)
    rng = np.random.default_rng(21)
    spec = W.front_spec(k=0.0, M=0.1, kappa=1.0, eps=1.0, gamma=1.0, DA=0.0, DB=0.0, DC=0.0, dt=0.005)
    spec.stencil = stencil
    spec.bc[0][4] = (MIRROR, 0.0)
    spec.bc[2] = [(GHOST, 1.0), (GHOST, -0.5), (PERIODIC, 0.0), (PERIODIC, 0.0), (GHOST, 0.25), (MIRROR, 0.0)]
    C0 = rng.uniform(-1, 1, shape)
    zero = np.zeros(shape)
    out = oracle.run(spec, [zero, zero, C0], 20)[2]
    assert abs(math.fsum(out.ravel()) - math.fsum(C0.ravel())) < 1e-12 * C0.size
    assert np.max(np.abs(out - C0)) > 1e-3          # the step did move C


@pytest.mark.parametrize("axes", [(0, 1), (0, 2), (1, 2)])
@pytest.mark.parametrize("h", [1.0, 2.0])
def test_stencil19_edge_ghost_takes_first_axis(oracle, axes, h):
    """An edge neighbour of the 19-point stencil that leaves the grid through
    two faces with different fixed ghost values takes the value of the first
    of the two axes in x, y, z order (the reading of the edge ghosts of
    section 4.1).  Uniform c0, low faces of axes a < b fixed at ga, gb: at a
    cell on both low faces, inside along the third axis, the stencil of
    Eq. (4) sums 2 (ga + gb) from the faces and 4 ga + 3 gb from the edges
    (the shared edge counted with ga), so
        Lap = D/(6h^2) (6 ga + 5 gb - 11 c0)."""
    shape = (6, 6, 6)
    c0, ga, gb, D, dt = 0.25, 1.5, -2.0, 1.0, 0.0625 * h * h
    bc = [(MIRROR, 0.0)] * 6
    bc[2 * axes[0]] = (GHOST, ga)
    bc[2 * axes[1]] = (GHOST, gb)
    spec = ModelSpec("diffusion", 1, dt, h, [[D] * 3], [bc], stencil=19)
    out = oracle.run(spec, [np.full(shape, c0)], 1)[0]
    idx = [slice(1, -1)] * 3          # inside along the third axis
    idx[2 - axes[0]] = 0
    idx[2 - axes[1]] = 0
    expect = c0 + dt * D / (6 * h * h) * (6 * ga + 5 * gb - 11 * c0)
    got = out[tuple(idx)]
    assert got.size == 4
    assert np.allclose(got, expect, rtol=0, atol=1e-14)


# ------------------------------------------------------------------ P7

def test_brusselator_uniform_is_scalar_ode(oracle):
    """A uniform field has zero Laplacian, so each cell follows the scalar
    forward-Euler recurrence of the Brusselator kinetics."""
    spec = W.brusselator_spec(kind=MIRROR)
    a, b, dt = spec.params["a"], spec.params["b"], spec.dt
    shape = (3, 4, 5)
    u, v = 1.0, 2.0
    out = oracle.run(spec, [np.full(shape, u), np.full(shape, v)], 60)
    for _ in range(60):
        u, v = u + dt * (a - (b + 1) * u + u * u * v), v + dt * (b * u - u * u * v)
    assert np.allclose(out[0], u, rtol=1e-13, atol=0)
    assert np.allclose(out[1], v, rtol=1e-13, atol=0)


def test_brusselator_fixed_point(oracle):
    w = W.make_workload("brusselator256", shape=(4, 5, 6))
    a, b = w.spec.params["a"], w.spec.params["b"]
    out = oracle.run(w.spec, [np.full(w.shape, a), np.full(w.shape, b / a)], 100)
    assert np.max(np.abs(out[0] - a)) < 1e-12 and np.max(np.abs(out[1] - b / a)) < 1e-12


def test_front_uniform_is_scalar_ode(oracle):
    spec = W.front_spec(k=0.7)
    spec.bc[0][4] = (MIRROR, 0.0)            # no held layer: fully uniform
    shape = (4, 3, 5)
    A, B, Cc = 0.8, 0.6, -0.3
    out = oracle.run(spec, [np.full(shape, A), np.full(shape, B), np.full(shape, Cc)], 40)
    for _ in range(40):
        r = 0.7 * A * B
        A, B, Cc = A - spec.dt * r, B - spec.dt * r, Cc + spec.dt * r
    for f, v in zip(out, (A, B, Cc)):
        assert np.allclose(f, v, rtol=1e-13, atol=1e-15)


def pollutant_spec(shape, ns=4, K=(0.0, 0.0, 0.0), wind=0.0, decay=0.0, kab=0.0,
                   dt=0.1, xkind=PERIODIC, sources=None, h=1.0):
    nz = shape[0]
    bc = uniform_bc(ns, MIRROR)
    for s in range(ns):
        bc[s][0] = (xkind, 0.0)
        bc[s][1] = (xkind if xkind == PERIODIC else MIRROR, 0.0)
    wind = np.full(nz, float(wind)) if np.isscalar(wind) else np.asarray(wind, float)
    src = sources or (np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros(0))
    return ModelSpec("pollutant", ns, dt, h, [list(K)] * ns, bc,
                     {"decay": decay, "kab": kab}, wind=wind, sources=src)


def test_pollutant_uniform_decay_and_coupling(oracle):
    """Uniform fields, periodic x: c_A, c_B follow a 2x2 linear recurrence,
    the other species decay by (1 - lambda dt)^n."""
    shape = (3, 4, 6)
    lam, kab, dt, n = 0.05, 0.2, 0.1, 30
    spec = pollutant_spec(shape, K=(0.5, 0.5, 0.1), wind=1.0, decay=lam, kab=kab, dt=dt)
    init = [1.0, 0.5, 2.0, 3.0]
    out = oracle.run(spec, [np.full(shape, v) for v in init], n)
    Mx = np.array([[1 - dt * (lam + kab), 0], [dt * kab, 1 - dt * lam]])
    ab = np.linalg.matrix_power(Mx, n) @ np.array(init[:2])
    expect = [ab[0], ab[1], init[2] * (1 - lam * dt) ** n, init[3] * (1 - lam * dt) ** n]
    for f, v in zip(out, expect):
        assert np.allclose(f, v, rtol=1e-13, atol=0)


def test_pollutant_isolated_source_accumulates(oracle):
    shape = (3, 4, 5)
    cell = (2 * 4 + 1) * 5 + 3
    src = (np.array([cell, cell, 7], np.int64), np.array([1, 1, 2], np.int32),
           np.array([10.0, 2.5, 4.0]))
    spec = pollutant_spec(shape, sources=src, dt=0.25)
    out = oracle.run(spec, [np.zeros(shape)] * 4, 12)
    exp1 = np.zeros(shape)
    exp1.ravel()[cell] = 12 * 0.25 * 12.5
    exp2 = np.zeros(shape)
    exp2.ravel()[7] = 12 * 0.25 * 4.0
    assert np.array_equal(out[0], np.zeros(shape)) and np.array_equal(out[3], np.zeros(shape))
    assert np.allclose(out[1], exp1, rtol=1e-14, atol=0)
    assert np.allclose(out[2], exp2, rtol=1e-14, atol=0)


# ------------------------------------------------------------------ P8

def test_brusselator_linearised_mode(oracle):
    """A small periodic mode about (a, b/a) evolves by the matrix
    I + dt (J - Lambda diag(Du, Dv)), J the kinetics' Jacobian there."""
    spec = W.brusselator_spec()
    a, b, dt = spec.params["a"], spec.params["b"], spec.dt
    Du, Dv = spec.K[0][0], spec.K[1][0]
    shape = (8, 10, 12)
    nz, ny, nx = shape
    k, j, i = grid_idx(shape)
    q = (1, 2, 3)
    mode = np.cos(2 * np.pi * (q[0] * k / nz + q[1] * j / ny + q[2] * i / nx))
    Lam = 4 * (np.sin(np.pi * q[0] / nz) ** 2 + np.sin(np.pi * q[1] / ny) ** 2
               + np.sin(np.pi * q[2] / nx) ** 2)
    eps, n = 1e-7, 50
    out = oracle.run(spec, [a + eps * mode, b / a + 0.5 * eps * mode], n)
    J = np.array([[b - 1, a * a], [-b, -a * a]])
    Mx = np.eye(2) + dt * (J - Lam * np.diag([Du, Dv]))
    pred = np.linalg.matrix_power(Mx, n) @ np.array([1.0, 0.5])
    proj = [np.sum((out[0] - a) * mode) / np.sum(mode * mode) / eps,
            np.sum((out[1] - b / a) * mode) / np.sum(mode * mode) / eps]
    assert np.allclose(proj, pred, rtol=2e-6, atol=0)


# ------------------------------------------------------------------ P9

def test_cahn_hilliard_linear_mode_factor(oracle):
    """With the cubic coefficient 0 and no reaction, a cosine mode of C
    is multiplied by 1 + dt M (eps Lam - kappa Lam^2) per step, Lam the
    Laplacian eigenvalue magnitude; the mean stays put."""
    shape = (6, 8, 10)
    nz, ny, nx = shape
    M, kappa, eps, dt, n = 0.1, 1.3, 0.7, 0.01, 40
    spec = W.front_spec(k=0.0, M=M, kappa=kappa, eps=eps, gamma=0.0, dt=dt)
    spec.bc[0][4] = (MIRROR, 0.0)
    vx, lx = mode_1d(MIRROR, nx, 3, 1.0)
    vy, ly = mode_1d(MIRROR, ny, 1, 1.0)
    vz, lz = mode_1d(MIRROR, nz, 2, 1.0)
    mode = vz[:, None, None] * vy[None, :, None] * vx[None, None, :]
    Lam = -(lx + ly + lz)
    g = 1 + dt * M * (eps * Lam - kappa * Lam**2)
    C0 = 0.25 + 0.1 * mode
    out = oracle.run(spec, [np.zeros(shape), np.zeros(shape), C0], n)
    assert np.max(np.abs(out[2] - (0.25 + 0.1 * g**n * mode))) < 1e-14


# ------------------------------------------------------------------ P10

@pytest.mark.parametrize("h", [1.0, 2.0])
def test_upwind_unit_cfl_is_exact_shift(oracle, h):
    """u dt / h = 1 moves every value exactly one cell downwind per step."""
    shape = (3, 4, 9)
    rng = np.random.default_rng(5)
    c0 = rng.integers(-50, 50, shape).astype(float)
    spec = pollutant_spec(shape, ns=1, wind=4.0 * h, dt=0.25, h=h)
    out = oracle.run(spec, [c0], 5)[0]
    assert np.array_equal(out, np.roll(c0, 5, axis=2))


def test_upwind_fourier_factor(oracle):
    """Constant wind, periodic x: a harmonic exp(i theta x) is multiplied by
    1 - nu (1 - exp(-i theta)) per step, nu = u dt / h."""
    shape = (2, 3, 16)
    nx = shape[2]
    theta, nu, n = 2 * np.pi * 3 / nx, 0.3, 20
    x = np.arange(nx)
    c0 = np.broadcast_to(np.cos(theta * x + 0.4), shape).copy()
    h = 1.5
    spec = pollutant_spec(shape, ns=1, wind=nu * h / 0.1, dt=0.1, h=h)
    out = oracle.run(spec, [c0], n)[0]
    A = (1 - nu * (1 - np.exp(-1j * theta))) ** n
    expect = np.real(A * np.exp(1j * (theta * x + 0.4)))
    assert np.max(np.abs(out - expect[None, None, :])) < 1e-14


def test_pollutant_mass_budget(oracle):
    """One step of the full pollutant model: the change of each species'
    total is exactly dt times (sources - decay - outflow through x+ by the
    wind - diffusive loss through the clean-inflow ghost at x-, -/+ the A->B
    transfer); no-flux y and z faces contribute nothing."""
    w = W.make_workload("pollutant512", shape=(6, 5, 8))
    rng = np.random.default_rng(9)
    fields = [rng.uniform(0, 1, w.shape) for _ in range(4)]
    spec = w.spec
    out = oracle.run(spec, fields, 1)
    dt, h = spec.dt, spec.h
    lam, kab = spec.params["decay"], spec.params["kab"]
    u = spec.wind[:, None]
    for s in range(4):
        Kx = spec.K[s][0]
        c = fields[s]
        flux = np.sum(-u * c[:, :, -1] / h) - Kx / h**2 * np.sum(c[:, :, 0])
        e = sum(r for cell, sp, r in zip(*spec.sources) if sp == s)
        change = flux - lam * np.sum(c) + e
        if s == 0:
            change -= kab * np.sum(fields[0])
        if s == 1:
            change += kab * np.sum(fields[0])
        got = math.fsum(out[s].ravel()) - math.fsum(c.ravel())
        assert abs(got - dt * change) < 1e-12 * max(1.0, np.sum(np.abs(c)))


# ------------------------------------------------------------------ P11

def test_held_layer_matches_1d_recurrence(oracle):
    """Fields uniform in x and y reduce to a 1D explicit heat recurrence with
    a held end (z=0) and a mirror end (z=nz-1)."""
    shape = (9, 3, 4)
    nz = shape[0]
    D, dt, n, held = 1.0, 0.1, 30, 1.0
    spec = diff_spec([D] * 3, dt)
    spec.bc[0][4] = (HELD, held)
    prof = np.linspace(0.0, 0.3, nz)
    c0 = np.broadcast_to(prof[:, None, None], shape).copy()
    out = oracle.run(spec, [c0], n)[0]
    p = prof.copy()
    for _ in range(n):
        q = p.copy()
        q[0] = held
        for kz in range(1, nz):
            up = p[kz + 1] if kz + 1 < nz else p[kz]
            dn = held if kz - 1 == 0 else p[kz - 1]
            q[kz] = p[kz] + dt * D * (up + dn - 2 * p[kz])
        p = q
    assert np.allclose(out, p[:, None, None], rtol=0, atol=1e-15)


def test_held_layer_mode_factor(oracle):
    """Held value 0 at z=0, mirror at z=nz-1: sin(theta k) with
    theta = pi (2q+1) / (2 nz - 1) is an exact eigenvector."""
    shape = (10, 2, 3)
    nz = shape[0]
    dt, n = 0.15, 20
    spec = diff_spec([1.0] * 3, dt)
    spec.bc[0][4] = (HELD, 0.0)
    theta = np.pi * 3 / (2 * nz - 1)
    v = np.sin(theta * np.arange(nz))
    g = 1 - dt * 4 * np.sin(theta / 2) ** 2
    out = oracle.run(spec, [np.broadcast_to(v[:, None, None], shape).copy()], n)[0]
    assert np.max(np.abs(out - g**n * v[:, None, None])) < 1e-14


# ------------------------------------------------------------------ P12

def test_periodic_shift_invariance(oracle):
    w = W.make_workload("brusselator256", shape=(6, 7, 8))
    sh = (2, 3, 5)
    out = oracle.run(w.spec, w.fields, 10)
    rolled = oracle.run(w.spec, [np.roll(f, sh, axis=(0, 1, 2)) for f in w.fields], 10)
    for a, b in zip(out, rolled):
        assert np.array_equal(np.roll(a, sh, axis=(0, 1, 2)), b)


# ------------------------------------------------------------------ reduce

def test_reduce_mass_energy(oracle):
    f = np.random.default_rng(1).uniform(-1, 2, (5, 6, 7))
    m, e = oracle.reduce(f, h=0.5)
    assert abs(m - math.fsum(f.ravel()) * 0.125) < 1e-13
    assert abs(e - math.fsum((f * f).ravel()) * 0.125) < 1e-13


# ------------------------------------------------------------------ P12
# The rest of Table 1: the Turing model, redissolution in the front model
# and the atmospheric wind.

def turing_spec(stencil=7, dt=5e-4, h=6.2e-3, D=(5e-5, 5e-3)):
    return ModelSpec("turing", 2, dt, h, [[D[0]] * 3, [D[1]] * 3], uniform_bc(2, MIRROR),
                     {"alpha": 0.5, "beta": 0.09, "gamma": 26.0}, stencil=stencil)


def turing_fixed_point(alpha=0.5, beta=0.09):
    """Homogeneous steady state: c1 - c1^3 - c2 = 0 and c1 - alpha c2 - beta = 0
    give alpha c1^3 + (1 - alpha) c1 - beta = 0 (one real root)."""
    r = np.roots([alpha, 0.0, 1.0 - alpha, -beta])
    c1 = float(np.real(r[np.abs(np.imag(r)) < 1e-12][0]))
    return c1, c1 - c1**3


@pytest.mark.parametrize("stencil", [7, 19])
def test_turing_fixed_point_is_steady(oracle, stencil):
    c1, c2 = turing_fixed_point()
    shape = (4, 5, 6)
    out = oracle.run(turing_spec(stencil), [np.full(shape, c1), np.full(shape, c2)], 40)
    assert np.max(np.abs(out[0] - c1)) < 1e-14 and np.max(np.abs(out[1] - c2)) < 1e-14


def laplacian_symbol(lams, h, stencil):
    """Eigenvalue of the 7- or 19-point Laplacian (per unit coefficient) on a
    separable mode whose 1D eigenvalues are lams; the 19-point one follows
    from v(i-1) + v(i+1) = s v(i), s = 2 + h^2 lambda, and Eq. (4)'s weights."""
    if stencil == 7:
        return sum(lams)
    s = [2.0 + h * h * l for l in lams]
    return (-24.0 + 2.0 * sum(s) + s[0] * s[1] + s[0] * s[2] + s[1] * s[2]) / (6.0 * h * h)


@pytest.mark.parametrize("stencil", [7, 19])
def test_turing_linearised_mode(oracle, stencil):
    """A small no-flux cosine mode about the steady state evolves by
    I + dt (J + Lam diag(D1, D2)) per step: J the Jacobian of Table 1's
    kinetics there, Lam the Laplacian's eigenvalue on the mode."""
    spec = turing_spec(stencil)
    c1, c2 = turing_fixed_point()
    al, ga, dt, h = 0.5, 26.0, spec.dt, spec.h
    shape = (6, 7, 8)
    nz, ny, nx = shape
    vx, lx = mode_1d(MIRROR, nx, 3, h)
    vy, ly = mode_1d(MIRROR, ny, 2, h)
    vz, lz = mode_1d(MIRROR, nz, 1, h)
    mode = vz[:, None, None] * vy[None, :, None] * vx[None, None, :]
    Lam = laplacian_symbol([lx, ly, lz], h, stencil)
    J = np.array([[1.0 - 3.0 * c1 * c1, -1.0], [ga, -ga * al]])
    G = np.eye(2) + dt * (J + Lam * np.diag([spec.K[0][0], spec.K[1][0]]))
    eps, n = 1e-7, 30
    out = oracle.run(spec, [c1 + eps * mode, c2 + 0.5 * eps * mode], n)
    pred = np.linalg.matrix_power(G, n) @ np.array([1.0, 0.5])
    proj = [np.sum((out[0] - c1) * mode) / np.sum(mode * mode) / eps,
            np.sum((out[1] - c2) * mode) / np.sum(mode * mode) / eps]
    assert np.allclose(proj, pred, rtol=2e-6, atol=0)
    # diffusion matters here: the same map without it predicts otherwise
    G0 = np.eye(2) + dt * J
    assert not np.allclose(proj, np.linalg.matrix_power(G0, n) @ np.array([1.0, 0.5]), rtol=1e-3)


@pytest.mark.parametrize("stencil", [7, 19])
def test_front_redissolution_budget(oracle, stencil):
    """With no-flux faces every Laplacian sums to zero, so one step changes
    sum(B + C) by exactly -dt k2 sum(A C) (redissolution removes C, the
    precipitation reaction moves B into C) and keeps sum(A - 2B - C)."""
    shape = (5, 6, 7)
    rng = np.random.default_rng(12)
    A, B, Cc = (rng.uniform(0.1, 1.0, shape) for _ in range(3))
    k1, k2, dt = 0.2, 0.3, 0.01
    spec = ModelSpec("front_ch", 3, dt, 1.0, [[1.0] * 3, [0.5] * 3, [0.0] * 3], uniform_bc(3, MIRROR),
                     {"k": k1, "k2": k2, "M": 1.0, "kappa": 1.0, "eps": 1.0, "gamma": 1.0},
                     stencil=stencil)
    out = oracle.run(spec, [A, B, Cc], 1)
    d_bc = (out[1] + out[2]).sum() - (B + Cc).sum()
    assert abs(d_bc - (-dt * k2 * np.sum(A * Cc))) < 1e-12 * abs(d_bc)
    inv0 = (A - 2 * B - Cc).sum()
    out = oracle.run(spec, [A, B, Cc], 6)
    assert abs((out[0] - 2 * out[1] - out[2]).sum() - inv0) < 1e-12 * np.sum(np.abs(A) + 2 * B + Cc)


def atmos_spec(shape, ux=0.0, uy=0.0, uz=0.0, T=0.0, t0=0.0, K=0.0, dt=0.5, h=1.0, bc=None,
               sources=None, stencil=7):
    return ModelSpec("atmos", 1, dt, h, [[K] * 3], bc if bc is not None else uniform_bc(1, MIRROR),
                     {"ux": ux, "uy": uy, "uz": uz, "uz_period": T, "t0": t0},
                     sources=sources, stencil=stencil)


def test_atmos_unit_cfl_is_exact_shift_on_every_axis(oracle):
    """|u| dt / h = 1 on one axis moves every value exactly one cell
    downwind per step, whichever way the wind blows; the vertical wind of
    Table 1, u_z sin(t / T), blows down at t = -pi T / 2 and up at +pi T / 2."""
    shape = (5, 6, 7)
    rng = np.random.default_rng(8)
    c0 = rng.integers(-50, 50, shape).astype(float)
    per = [(PERIODIC, 0.0)] * 6
    out = oracle.run(atmos_spec(shape, ux=2.0, bc=[per]), [c0], 3)[0]
    assert np.array_equal(out, np.roll(c0, 3, axis=2))
    out = oracle.run(atmos_spec(shape, uy=-2.0, bc=[per]), [c0], 3)[0]
    assert np.array_equal(out, np.roll(c0, -3, axis=1))
    down = oracle.run(atmos_spec(shape, uz=2.0, T=1.0, t0=-math.pi / 2, bc=[per]), [c0], 1)[0]
    assert np.array_equal(down, np.roll(c0, -1, axis=0))
    up = oracle.run(atmos_spec(shape, uz=2.0, T=1.0, t0=math.pi / 2, bc=[per]), [c0], 1)[0]
    assert np.array_equal(up, np.roll(c0, 1, axis=0))


@pytest.mark.parametrize("stencil", [7, 19])
def test_atmos_mass_budget(oracle, stencil):
    """No-flux (mirror) faces: diffusion sums to zero and the upwind sums
    telescope, so one step changes the total by exactly
    dt (sum E - sum_d (u_d / h) sum over lines along d of (c_last - c_first)),
    for either sign of each wind component."""
    shape = (6, 7, 8)
    rng = np.random.default_rng(31)
    c0 = rng.uniform(0.0, 2.0, shape)
    nz, ny, nx = shape
    cells = np.array([(2 * ny + 3) * nx + 4, (4 * ny + 1) * nx + 6], np.int64)
    rates = np.array([10.0, 2.5])
    ux, uy, uz, T, t0, dt, h = 0.3, -0.2, 0.4, 3.0, 1.0, 0.05, 1.5
    spec = atmos_spec(shape, ux, uy, uz, T, t0, K=0.7, dt=dt, h=h, stencil=stencil,
                      sources=(cells, np.zeros(2, np.int32), rates))
    out = oracle.run(spec, [c0], 1)[0]
    u = [ux, uy, uz * math.sin(t0 / T)]
    flux = sum(u[d] / h * np.sum(np.take(c0, -1, axis=2 - d) - np.take(c0, 0, axis=2 - d))
               for d in range(3))
    expect = dt * (rates.sum() - flux)
    assert abs((out.sum() - c0.sum()) - expect) < 1e-12 * c0.sum()


# ------------------------------------------------------------------ P13
# Strong-stability-preserving Runge-Kutta steps built from Euler steps.

RK_FACTOR = {
    "euler": lambda z: 1 + z,
    "rk2": lambda z: 1 + z + z * z / 2,
    "rk3": lambda z: 1 + z + z * z / 2 + z**3 / 6,
}


@pytest.mark.parametrize("integrator", ["rk2", "rk3"])
@pytest.mark.parametrize("stencil", [7, 19])
@pytest.mark.parametrize("kinds", [(MIRROR, MIRROR, MIRROR), (PERIODIC, MIRROR, GHOST)])
def test_rk_fourier_mode_factor(oracle, integrator, stencil, kinds):
    """On a linear problem each stage is a polynomial in dt L, so a discrete
    Fourier mode is multiplied per step by the method's stability polynomial
    R(z) at z = dt lambda: 1 + z + z^2/2 (order 2), + z^3/6 (order 3)."""
    shape = (5, 6, 11)
    nz, ny, nx = shape
    h, D, dt, n = 1.3, 0.6, 0.2, 15
    vx, lx = mode_1d(kinds[0], nx, 2, h)
    vy, ly = mode_1d(kinds[1], ny, 1, h)
    vz, lz = mode_1d(kinds[2], nz, 3, h)
    mode = vz[:, None, None] * vy[None, :, None] * vx[None, None, :]
    z = dt * D * laplacian_symbol([lx, ly, lz], h, stencil)
    spec = ModelSpec("diffusion", 1, dt, h, [[D] * 3], axis_bc(kinds), stencil=stencil, integrator=integrator)
    out = oracle.run(spec, [mode], n)[0]
    assert np.max(np.abs(out - RK_FACTOR[integrator](z) ** n * mode)) < 1e-14


@pytest.mark.parametrize("integrator,order", [("euler", 1), ("rk2", 2), ("rk3", 3)])
def test_rk_order_of_accuracy(oracle, integrator, order):
    """Against the exact decay exp(lambda T) of one mode of the semi-discrete
    problem, halving dt divides the error at a fixed time by about 2^order."""
    shape = (4, 4, 16)
    vx, lx = mode_1d(PERIODIC, 16, 1, 1.0)
    mode = np.broadcast_to(vx, shape).copy()
    D, T = 1.0, 2.0
    errs = []
    for n in (10, 20, 40):
        spec = ModelSpec("diffusion", 1, T / n, 1.0, [[D] * 3], axis_bc((PERIODIC, MIRROR, MIRROR)),
                         integrator=integrator)
        out = oracle.run(spec, [mode], n)[0]
        errs.append(np.max(np.abs(out - np.exp(D * lx * T) * mode)))
    for a, b in zip(errs, errs[1:]):
        assert 0.85 * 2**order < a / b < 1.15 * 2**order, errs


@pytest.mark.parametrize("integrator", ["rk2", "rk3"])
def test_rk_keeps_held_layers_and_rejects_clocked_wind(oracle, integrator):
    shape = (5, 6, 7)
    rng = np.random.default_rng(3)
    faces = [(HELD, 1.5), (MIRROR, 0), (GHOST, 0.25), (MIRROR, 0), (MIRROR, 0), (HELD, -0.5)]
    spec = ModelSpec("diffusion", 1, 0.1, 1.0, [[1.0] * 3], [faces], integrator=integrator)
    c0 = rng.uniform(0, 1, shape)
    c0[:, :, 0] = 1.5
    c0[-1, :, :] = -0.5
    c0[-1, :, 0] = 1.5                      # x- decides where the two held faces meet
    out = oracle.run(spec, [c0], 7)[0]
    assert np.all(np.abs(out[:, :, 0] - 1.5) < 1e-15) and np.all(np.abs(out[-1, :, 1:] + 0.5) < 1e-15)
    a = ModelSpec("atmos", 1, 0.1, 1.0, [[0.1] * 3], uniform_bc(1, MIRROR),
                  {"ux": 1.0, "uy": 0.0, "uz": 1.0, "uz_period": 2.0}, integrator=integrator)
    with pytest.raises(ValueError):
        oracle.run(a, [c0], 1)


# ------------------------------------------------------------------ P14
# Counter-based random bits for stochastic rounding (oracle side).

def test_philox_known_answers():
    """Philox-2x32-10 against the known-answer vectors of its authors'
    reference distribution."""
    from oracle.stochastic import philox2x32_10
    cases = [((0x00000000, 0x00000000), 0x00000000, (0xff1dae59, 0x6cd10df2)),
             ((0xffffffff, 0xffffffff), 0xffffffff, (0x2c3f628b, 0xab4fd7ad)),
             ((0x243f6a88, 0x85a308d3), 0x13198a2e, (0xdd7ce038, 0xf62a4c12))]
    for (c0, c1), k, want in cases:
        got = philox2x32_10(c0, c1, k)
        assert (int(got[0]), int(got[1])) == want


def test_bf16_stochastic_rounding_is_unbiased():
    """Rounding up happens for exactly the random draws at or above 2^16
    minus the discarded bits, so over all 2^16 draws the mean is x."""
    from oracle.stochastic import bf16_stochastic
    x = np.float32(1.0 - 2.0**-10)          # 3/4 of the way from 1 - 2^-8 to 1
    r = np.arange(65536, dtype=np.uint32)
    y = bf16_stochastic(np.full(65536, x), r)
    assert set(np.unique(y).tolist()) == {1.0 - 2.0**-8, 1.0}
    assert np.count_nonzero(y == 1.0) == 49152
    assert np.mean(y.astype(np.float64)) == float(x)
    z = bf16_stochastic(np.float32([0.5, -3.0]), np.uint32([65535, 65535]))
    assert z.tolist() == [0.5, -3.0]         # representable values never move


def test_random16_positions_are_uniform_and_independent():
    """The four 16-bit draws taken from one Philox-2x32-10 call (elements 4c
    .. 4c+3) are each uniform on 0 .. 2^16-1 and uncorrelated with their
    neighbours, over 2^18 consecutive elements of one step."""
    from oracle.stochastic import random16
    e = np.arange(1 << 18, dtype=np.uint64)
    r = random16(e, 7, 20240611, 2).astype(np.float64)
    n = r.size // 4
    for q in range(4):
        x = r[q::4]
        assert abs(x.mean() - 32767.5) < 5 * 18918.6 / math.sqrt(n)
        counts = np.bincount((x // 4096).astype(int), minlength=16)
        chi2 = np.sum((counts - n / 16) ** 2 / (n / 16))
        assert chi2 < 50.0                                  # 15 dof: p < 1e-5
    c = np.corrcoef(r[:-1], r[1:])[0, 1]
    assert abs(c) < 5 / math.sqrt(r.size)
    # another step gives other bits for the same elements
    assert np.mean(random16(e[:4096], 8, 20240611, 2) == r[:4096]) < 0.01
