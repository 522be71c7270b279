/*
 * rd_oracle.h -- FP64 CPU oracle for the explicit method-of-lines
 * reaction-diffusion step (Molnar, Izsak, Meszaros, Lagzi, "Simulation of
 * reaction-diffusion processes in three dimensions using CUDA").
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * reference that the HIP path is checked against.  Only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * What it computes (section 2, Eqs. (2) and (5); Table 3):
 *   c_s(t+dt) = c_s(t) + dt * [ L_s(c_s) + A_s(c_s) + R_s(c(t)) + E_s ]
 * with L_s the 7-point Laplacian (the "more commonly used seven-point
 * stencil" mentioned beside Eqs. (3)-(4)), allowing a different coefficient
 * per axis, or the 19-point Laplacian of Eqs. (3)-(4) (isotropic
 * coefficient), A_s the first-order upwind advection term of section 4.1, R_s the
 * reaction term evaluated at the old time level, and E_s point emissions
 * (Table 1, advection-diffusion row).  Boundary values are fixed before each
 * step from the boundary conditions (section 4.1, Table 3 lines 4-5).
 *
 * Grid convention: every one of the nx*ny*nz cells is an unknown; a value
 * one step outside the grid is a virtual ghost given by the face's rule:
 *   OR_MIRROR    ghost = the adjacent cell (no-flux, zero-gradient, outflow)
 *   OR_PERIODIC  ghost = the cell at the other end of the axis
 *   OR_GHOST     ghost = a fixed value (e.g. clean inflow, 0)
 *   OR_HELD      the face's own layer of cells is held at a fixed value and
 *                never updated (a Dirichlet layer); its ghost is that value.
 * A cell lying on several held faces takes the value of the first such face
 * in the order x-, x+, y-, y+, z-, z+.  A 19-point edge neighbour may lie
 * outside along two axes (the edge ghosts of section 4.1): the rule of the
 * first such axis in the order x, y, z applies first (a mirror or periodic
 * rule moves that coordinate inside and the next axis is resolved).
 *
 * Arrays: one species is a float64 array [nz][ny][nx] (x fastest), as in the
 * paper's C[Depth][Height][Width]; a state is ns such arrays back to back.
 */
#ifndef RD_ORACLE_H
#define RD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_SPECIES 4

enum { OR_MIRROR = 0, OR_PERIODIC = 1, OR_GHOST = 2, OR_HELD = 3 };
enum { OR_DIFFUSION = 0, OR_BRUSSELATOR = 1, OR_FRONT_CH = 2, OR_POLLUTANT = 3,
       OR_TURING = 4, OR_ATMOS = 5 };

/* Model constants in p[]:
 *   OR_BRUSSELATOR  p[0]=a  p[1]=b
 *       R_u = a - (b+1) u + u^2 v ,  R_v = b u - u^2 v
 *   OR_FRONT_CH     p[0]=k  p[1]=M  p[2]=kappa  p[3]=eps  p[4]=gamma  p[5]=k2
 *       species A, B, C;  r = k A B ,  q = k2 A C  (redissolution)
 *       R_A = -r - q ,  R_B = -r ,  R_C = r - q + M Lap(mu),
 *       mu = gamma C^3 - eps C - kappa Lap(C)
 *     (Table 1, third row: k = k_1, k2 = k_2, -lambda Lap(eps c - gamma c^3 + sigma Lap c) with
 *      lambda = M and sigma = kappa; the biharmonic part is the Laplacian
 *      taken twice with boundary values re-applied in between, section 4.1.
 *      mu's ghosts are mirror on every face.)
 *   OR_POLLUTANT    p[0]=decay lambda  p[1]=k_AB (species 0 -> species 1)
 *       A_s = -u(z) (c_s(i) - c_s(i-1)) / h     (upwind, u >= 0 along +x)
 *       R_s = -lambda c_s ;  R_0 -= k_AB c_0 ;  R_1 += k_AB c_0
 *   OR_TURING       p[0]=alpha  p[1]=beta  p[2]=gamma   (Table 1, second row)
 *       R_1 = c_1 - c_1^3 - c_2 ,  R_2 = gamma (c_1 - alpha c_2 - beta)
 *   OR_ATMOS        p[0]=u_x  p[1]=u_y  p[2]=u_z amplitude  p[3]=T  p[4]=t_0
 *       (Table 1, last row) a wind uniform in space, u = (u_x, u_y, u_z(t)),
 *       u_z(t) = p[2] sin(t / T) (p[2] itself when T = 0), t = t_0 + n dt at
 *       step n; A_s = sum over axes of the first-order upwind form of
 *       -u_d dc/dx_d (the difference on the side the wind comes from);
 *       E_s = point emissions (src_*); every species carried independently.
 */
typedef struct or_problem {
    int64_t nx, ny, nz;
    int32_t ns;
    int32_t model;
    double h;
    double dt;
    double K[OR_MAX_SPECIES][3];          /* per species, per axis x,y,z */
    int32_t bc_kind[OR_MAX_SPECIES][6];   /* faces x-,x+,y-,y+,z-,z+      */
    double bc_value[OR_MAX_SPECIES][6];
    double p[8];
    const double *wind;                   /* nz values (pollutant), else NULL */
    int64_t nsrc;                         /* point sources (pollutant, atmos) */
    const int64_t *src_cell;              /* linear index (k*ny + j)*nx + i   */
    const int32_t *src_species;
    const double *src_rate;
    int32_t stencil;                      /* 7, or 19 (needs K[s][0]=K[s][1]=K[s][2]) */
    int32_t integrator;                   /* OR_EULER (0 or 1), OR_RK2, OR_RK3 */
} or_problem;

/* Time integrators.  Forward Euler is Eq. (5); the others are the
 * strong-stability-preserving Runge-Kutta methods of order 2 (Heun) and 3
 * (Shu-Osher), built from Euler steps E(u) = u + dt F(u):
 *   OR_RK2:  u1 = E(c);  c' = c/2 + E(u1)/2
 *   OR_RK3:  u1 = E(c);  u2 = 3c/4 + E(u1)/4;  c' = c/3 + 2 E(u2)/3
 * (the paper notes that more accurate steppers exist, section 2).  Held
 * layers keep their value through every stage.  Models whose terms depend
 * on time (the atmospheric wind) take forward Euler only. */
enum { OR_EULER = 1, OR_RK2 = 2, OR_RK3 = 3 };

/* Advance `state` (ns*nz*ny*nx doubles) by nsteps explicit Euler steps in
 * place.  Returns 0, or -1 on a bad argument / allocation failure. */
int or_run(const or_problem *P, double *state, int64_t nsteps);

/* The Cahn-Hilliard chemical potential mu = gamma C^3 - eps C - kappa Lap(C)
 * of species 2 of `state`, for every cell (front model only). */
int or_mu(const or_problem *P, const double *state, double *mu);

/* FP64 mass sum(c) h^3 and energy sum(c^2) h^3 of one field. */
void or_reduce(int64_t nx, int64_t ny, int64_t nz, double h, const double *f,
               double out[2]);

/* Number of threads or_run uses. */
int or_threads(void);

/* Use n threads from now on (n >= 1; the paper's CPU baseline is one
 * thread); returns the number now in use. */
int or_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
