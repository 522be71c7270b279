/*
 * rd_oracle.c -- FP64 CPU oracle for the explicit reaction-diffusion step.
 *
 * TEST INFRASTRUCTURE ONLY (see rd_oracle.h): plain loops, one cell at a
 * time, every neighbour fetched through the ghost rule of its face.  The
 * OpenMP loop over z only splits independent cells between threads; each
 * cell's arithmetic is the same whatever the thread count.
 */
#include "rd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ ghosts */

/* Is cell (i,j,k) on a held layer of this field?  Faces are tried in the
 * order x-, x+, y-, y+, z-, z+ and the first held one decides. */
static int held_value(const int32_t kind[6], const double val[6],
                      int64_t nx, int64_t ny, int64_t nz,
                      int64_t i, int64_t j, int64_t k, double *v)
{
    const int on[6] = { i == 0, i == nx - 1, j == 0, j == ny - 1, k == 0, k == nz - 1 };
    for (int f = 0; f < 6; ++f) {
        if (kind[f] == OR_HELD && on[f]) {
            *v = val[f];
            return 1;
        }
    }
    return 0;
}

/* Value of a field at (i,j,k), where at most one coordinate may lie one cell
 * outside the grid (a 7-point neighbour never leaves along two axes).
 * Boundary values are set from the boundary conditions (section 4.1). */
static double sample(const double *f, int64_t nx, int64_t ny, int64_t nz,
                     const int32_t kind[6], const double val[6],
                     int64_t i, int64_t j, int64_t k)
{
    int face = -1;
    if (i < 0) face = 0;
    else if (i >= nx) face = 1;
    else if (j < 0) face = 2;
    else if (j >= ny) face = 3;
    else if (k < 0) face = 4;
    else if (k >= nz) face = 5;

    if (face < 0) {
        double v;
        if (held_value(kind, val, nx, ny, nz, i, j, k, &v)) return v;
        return f[(k * ny + j) * nx + i];
    }
    switch (kind[face]) {
    case OR_MIRROR:          /* ghost equals the adjacent (edge) cell */
        if (face == 0) i = 0;
        if (face == 1) i = nx - 1;
        if (face == 2) j = 0;
        if (face == 3) j = ny - 1;
        if (face == 4) k = 0;
        if (face == 5) k = nz - 1;
        return sample(f, nx, ny, nz, kind, val, i, j, k);
    case OR_PERIODIC:        /* ghost equals the cell at the other end */
        if (face == 0) i = nx - 1;
        if (face == 1) i = 0;
        if (face == 2) j = ny - 1;
        if (face == 3) j = 0;
        if (face == 4) k = nz - 1;
        if (face == 5) k = 0;
        return sample(f, nx, ny, nz, kind, val, i, j, k);
    case OR_GHOST:
    case OR_HELD:
    default:
        return val[face];
    }
}

/* 7-point Laplacian with per-axis coefficient:
 *   sum_d K_d (c[+e_d] + c[-e_d] - 2 c) / h^2           (section 2) */
static double laplacian(const double *f, int64_t nx, int64_t ny, int64_t nz,
                        const int32_t kind[6], const double val[6], double h,
                        const double K[3], int64_t i, int64_t j, int64_t k)
{
    const double c = sample(f, nx, ny, nz, kind, val, i, j, k);
    const double dx = sample(f, nx, ny, nz, kind, val, i - 1, j, k)
                    + sample(f, nx, ny, nz, kind, val, i + 1, j, k) - 2.0 * c;
    const double dy = sample(f, nx, ny, nz, kind, val, i, j - 1, k)
                    + sample(f, nx, ny, nz, kind, val, i, j + 1, k) - 2.0 * c;
    const double dz = sample(f, nx, ny, nz, kind, val, i, j, k - 1)
                    + sample(f, nx, ny, nz, kind, val, i, j, k + 1) - 2.0 * c;
    return (K[0] * dx + K[1] * dy + K[2] * dz) / (h * h);
}

/* 19-point Laplacian of Eqs. (3)-(4), isotropic coefficient D:
 *   D/(6h^2) * sum over the 3x3x3 block of T_pqr c[i+p][j+q][k+r]
 * with T = -24 at the centre, 2 at the six face neighbours, 1 at the twelve
 * edge neighbours (|p|+|q|+|r| = 2) and 0 at the eight corners. */
static double laplacian19(const double *f, int64_t nx, int64_t ny, int64_t nz,
                          const int32_t kind[6], const double val[6], double h,
                          double D, int64_t i, int64_t j, int64_t k)
{
    double sum = 0.0;
    for (int r = -1; r <= 1; ++r)
        for (int q = -1; q <= 1; ++q)
            for (int p = -1; p <= 1; ++p) {
                const int order = abs(p) + abs(q) + abs(r);
                const double T = order == 0 ? -24.0 : order == 1 ? 2.0 : order == 2 ? 1.0 : 0.0;
                if (T != 0.0)
                    sum += T * sample(f, nx, ny, nz, kind, val, i + p, j + q, k + r);
            }
    return D * sum / (6.0 * h * h);
}

/* The Laplacian the problem asks for (K: per-axis coefficients; the 19-point
 * form uses K[0]). */
static double lap_of(const or_problem *P, const double *f, const int32_t kind[6],
                     const double val[6], const double K[3], int64_t i, int64_t j, int64_t k)
{
    if (P->stencil == 19)
        return laplacian19(f, P->nx, P->ny, P->nz, kind, val, P->h, K[0], i, j, k);
    return laplacian(f, P->nx, P->ny, P->nz, kind, val, P->h, K, i, j, k);
}

/* ---------------------------------------------------------------- sources */

typedef struct { int64_t cell; int32_t species; double rate; } source_t;

static int cmp_source(const void *a, const void *b)
{
    const source_t *x = (const source_t *)a, *y = (const source_t *)b;
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    return x->species - y->species;
}

/* Sum of the emission rates of species s at `cell` (duplicates add up). */
static double emission(const source_t *src, int64_t n, int64_t cell, int s)
{
    int64_t lo = 0, hi = n;                 /* first index with src.cell >= cell */
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (src[mid].cell < cell) lo = mid + 1; else hi = mid;
    }
    double e = 0.0;
    for (int64_t q = lo; q < n && src[q].cell == cell; ++q)
        if (src[q].species == s) e += src[q].rate;
    return e;
}

/* ---------------------------------------------------------------- checks */

static int valid(const or_problem *P)
{
    if (!P || P->nx < 1 || P->ny < 1 || P->nz < 1) return 0;
    if (P->ns < 1 || P->ns > OR_MAX_SPECIES) return 0;
    if (P->model == OR_BRUSSELATOR && P->ns != 2) return 0;
    if (P->model == OR_FRONT_CH && P->ns != 3) return 0;
    if (P->model == OR_TURING && P->ns != 2) return 0;
    if (P->model < OR_DIFFUSION || P->model > OR_ATMOS) return 0;
    if (P->model == OR_POLLUTANT && !P->wind) return 0;
    if (P->stencil != 7 && P->stencil != 19) return 0;
    if (P->integrator < 0 || P->integrator > OR_RK3) return 0;
    if (P->integrator >= OR_RK2 && P->model == OR_ATMOS) return 0;
    if (P->stencil == 19)
        for (int s = 0; s < P->ns; ++s)
            if (P->K[s][1] != P->K[s][0] || P->K[s][2] != P->K[s][0]) return 0;
    for (int s = 0; s < P->ns; ++s)
        for (int a = 0; a < 3; ++a) {
            const int lo = P->bc_kind[s][2 * a], hi = P->bc_kind[s][2 * a + 1];
            if ((lo == OR_PERIODIC) != (hi == OR_PERIODIC)) return 0;
        }
    return 1;
}

/* ------------------------------------------------------------- one step */

static const int32_t MU_KIND[6] = { OR_MIRROR, OR_MIRROR, OR_MIRROR,
                                    OR_MIRROR, OR_MIRROR, OR_MIRROR };
static const double MU_VAL[6] = { 0, 0, 0, 0, 0, 0 };

/* mu = gamma C^3 - eps C - kappa Lap(C) on every cell, C = species 2, with
 * C's own boundary values (the first of the two Laplacian passes). */
static void chemical_potential(const or_problem *P, const double *C, double *mu)
{
    const int64_t nx = P->nx, ny = P->ny, nz = P->nz;
    const double kappa = P->p[2], eps = P->p[3], gamma = P->p[4];
    const double unit[3] = { 1.0, 1.0, 1.0 };
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const double c = sample(C, nx, ny, nz, P->bc_kind[2], P->bc_value[2], i, j, k);
                const double lap = lap_of(P, C, P->bc_kind[2], P->bc_value[2], unit, i, j, k);
                mu[(k * ny + j) * nx + i] = gamma * c * c * c - eps * c - kappa * lap;
            }
}

/* First-order upwind approximation of -u d(c)/d(axis) at (i, j, k): the
 * one-sided difference on the side the wind comes from (section 4.1). */
static double upwind(const or_problem *P, const double *f, const int32_t kind[6],
                     const double val[6], double u, int axis, int64_t i, int64_t j, int64_t k)
{
    const int64_t di = axis == 0, dj = axis == 1, dk = axis == 2;
    const double c = sample(f, P->nx, P->ny, P->nz, kind, val, i, j, k);
    if (u > 0.0)
        return -u * (c - sample(f, P->nx, P->ny, P->nz, kind, val, i - di, j - dj, k - dk)) / P->h;
    if (u < 0.0)
        return -u * (sample(f, P->nx, P->ny, P->nz, kind, val, i + di, j + dj, k + dk) - c) / P->h;
    return 0.0;
}

/* One forward Euler step (Eq. (5)) from `in` to `out` (Table 3 lines 4-9);
 * `t` is the time of the old level. */
static void step(const or_problem *P, const double *in, double *out, double *mu,
                 const source_t *src, int64_t nsrc, double t)
{
    const int64_t nx = P->nx, ny = P->ny, nz = P->nz, N = nx * ny * nz;
    const int ns = P->ns;
    const double dt = P->dt, h = P->h;
    const double unit[3] = { 1.0, 1.0, 1.0 };
    /* atmospheric wind at time t (Table 1, last row) */
    const double wind[3] = { P->p[0], P->p[1],
                             P->p[3] != 0.0 ? P->p[2] * sin(t / P->p[3]) : P->p[2] };

    if (P->model == OR_FRONT_CH)
        chemical_potential(P, in + 2 * N, mu);

#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t idx = (k * ny + j) * nx + i;
                double c[OR_MAX_SPECIES], rate[OR_MAX_SPECIES];
                for (int s = 0; s < ns; ++s) {
                    c[s] = sample(in + s * N, nx, ny, nz, P->bc_kind[s], P->bc_value[s], i, j, k);
                    rate[s] = lap_of(P, in + s * N, P->bc_kind[s], P->bc_value[s], P->K[s], i, j, k);
                }
                switch (P->model) {
                case OR_BRUSSELATOR: {
                    const double a = P->p[0], b = P->p[1], u = c[0], v = c[1];
                    rate[0] += a - (b + 1.0) * u + u * u * v;
                    rate[1] += b * u - u * u * v;
                    break;
                }
                case OR_FRONT_CH: {
                    const double r = P->p[0] * c[0] * c[1];
                    const double q = P->p[5] * c[0] * c[2];    /* redissolution A + C */
                    const double lap_mu = lap_of(P, mu, MU_KIND, MU_VAL, unit, i, j, k);
                    rate[0] += -r - q;
                    rate[1] += -r;
                    rate[2] += r - q + P->p[1] * lap_mu;
                    break;
                }
                case OR_TURING: {
                    const double u = c[0], v = c[1];
                    rate[0] += u - u * u * u - v;
                    rate[1] += P->p[2] * (u - P->p[0] * v - P->p[1]);
                    break;
                }
                case OR_ATMOS:
                    for (int s = 0; s < ns; ++s) {
                        for (int d = 0; d < 3; ++d)
                            rate[s] += upwind(P, in + s * N, P->bc_kind[s], P->bc_value[s], wind[d], d, i, j, k);
                        rate[s] += emission(src, nsrc, idx, s);
                    }
                    break;
                case OR_POLLUTANT: {
                    const double u = P->wind[k];
                    for (int s = 0; s < ns; ++s) {
                        const double left = sample(in + s * N, nx, ny, nz, P->bc_kind[s],
                                                   P->bc_value[s], i - 1, j, k);
                        rate[s] += -u * (c[s] - left) / h;     /* upwind, u >= 0 */
                        rate[s] += -P->p[0] * c[s];            /* first-order decay */
                        rate[s] += emission(src, nsrc, idx, s);
                    }
                    if (ns >= 2) {                             /* A -> B */
                        rate[0] -= P->p[1] * c[0];
                        rate[1] += P->p[1] * c[0];
                    }
                    break;
                }
                default:
                    break;
                }
                for (int s = 0; s < ns; ++s) {
                    double hv;
                    if (held_value(P->bc_kind[s], P->bc_value[s], nx, ny, nz, i, j, k, &hv))
                        out[s * N + idx] = hv;             /* held layer: not updated */
                    else
                        out[s * N + idx] = c[s] + dt * rate[s];
                }
            }
}

int or_run(const or_problem *P, double *state, int64_t nsteps)
{
    if (!valid(P) || !state || nsteps < 0) return -1;
    const int64_t N = P->nx * P->ny * P->nz;
    const size_t bytes = (size_t)P->ns * (size_t)N * sizeof(double);
    double *work = (double *)malloc(bytes);
    double *mu = P->model == OR_FRONT_CH ? (double *)malloc((size_t)N * sizeof(double)) : NULL;
    source_t *src = NULL;
    int64_t nsrc = 0;
    if (!work || (P->model == OR_FRONT_CH && !mu)) { free(work); free(mu); return -1; }
    if ((P->model == OR_POLLUTANT || P->model == OR_ATMOS) && P->nsrc > 0) {
        src = (source_t *)malloc((size_t)P->nsrc * sizeof(source_t));
        if (!src) { free(work); free(mu); return -1; }
        for (int64_t q = 0; q < P->nsrc; ++q) {
            src[q].cell = P->src_cell[q];
            src[q].species = P->src_species[q];
            src[q].rate = P->src_rate[q];
        }
        nsrc = P->nsrc;
        qsort(src, (size_t)nsrc, sizeof(source_t), cmp_source);
    }
    if (P->integrator >= OR_RK2) {
        /* two more stage arrays: u = E(c) and E(u) */
        double *u = (double *)malloc(bytes), *eu = (double *)malloc(bytes);
        if (!u || !eu) { free(u); free(eu); free(work); free(mu); free(src); return -1; }
        const size_t total = (size_t)P->ns * (size_t)N;
        for (int64_t n = 0; n < nsteps; ++n) {
            step(P, state, u, mu, src, nsrc, 0.0);          /* u1 = E(c)      */
            step(P, u, eu, mu, src, nsrc, 0.0);             /* E(u1)          */
            if (P->integrator == OR_RK2) {
                for (size_t q = 0; q < total; ++q) state[q] = 0.5 * state[q] + 0.5 * eu[q];
                continue;
            }
            for (size_t q = 0; q < total; ++q) u[q] = 0.75 * state[q] + 0.25 * eu[q];   /* u2 */
            step(P, u, eu, mu, src, nsrc, 0.0);             /* E(u2)          */
            for (size_t q = 0; q < total; ++q) state[q] = state[q] / 3.0 + 2.0 * eu[q] / 3.0;
        }
        free(u);
        free(eu);
        free(work);
        free(mu);
        free(src);
        return 0;
    }
    double *a = state, *b = work;
    for (int64_t n = 0; n < nsteps; ++n) {
        step(P, a, b, mu, src, nsrc, P->p[4] + (double)n * P->dt);
        double *t = a; a = b; b = t;            /* swap first and second arrays */
    }
    if (a != state) memcpy(state, a, bytes);
    free(work);
    free(mu);
    free(src);
    return 0;
}

int or_mu(const or_problem *P, const double *state, double *mu)
{
    if (!valid(P) || P->model != OR_FRONT_CH || !state || !mu) return -1;
    const int64_t N = P->nx * P->ny * P->nz;
    chemical_potential(P, state + 2 * N, mu);
    return 0;
}

void or_reduce(int64_t nx, int64_t ny, int64_t nz, double h, const double *f, double out[2])
{
    double m = 0.0, e = 0.0;
    const int64_t N = nx * ny * nz;
    for (int64_t q = 0; q < N; ++q) {
        m += f[q];
        e += f[q] * f[q];
    }
    out[0] = m * h * h * h;
    out[1] = e * h * h * h;
}

int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return or_threads();
}

int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
