/*
 * rd.h -- C ABI of the MI355X reaction-diffusion stepper (librdmi.so).
 *
 * The library advances 3D reaction-diffusion systems
 *     dc_s/dt = sum_d K_{s,d} d^2 c_s/dx_d^2 + A_s(c_s) + R_s(c) + E_s
 * on a uniform grid by the method of lines with forward Euler in time
 * (section 2, Eqs. (2) and (5) of Molnar, Izsak, Meszaros, Lagzi, "Simulation
 * of reaction-diffusion processes in three dimensions using CUDA"), using the
 * 7-point Laplacian the paper names beside its 19-point stencil (Eqs. (3)-(4)).
 * One step is one fused HIP kernel on gfx950 (two for the Cahn-Hilliard
 * model, whose biharmonic term is the Laplacian taken twice, section 4.1):
 * boundary values, Laplacian, advection, reaction and the Euler update all
 * happen in registers between one read and one write of each species.
 *
 * Conventions shared by every call:
 *   - A field is an array [nz][ny][nx], x contiguous (the paper's
 *     C[Depth][Height][Width], Tables 4-5).  Host and device buffers handed
 *     to the library are dense in that layout; internally rows are padded.
 *   - All nx*ny*nz cells are unknowns.  A neighbour one cell outside the grid
 *     is a virtual ghost given by the face's boundary rule (RD_BC_*), set
 *     before each step as in Table 3 lines 4-5.
 *   - Compute is FP32.  Fields may be stored as FP32, BF16 or FP16 (rounded to
 *     nearest even after each step); reductions accumulate in FP64.
 *   - Every call returns RD_OK (0) or a negative RD_E* code and never throws;
 *     rd_last_error() then gives a message (thread-local).  Invalid arguments
 *     are rejected before any device work.  Device faults surface as
 *     RD_EDEVICE at the next call that synchronises.
 *   - Calls on one grid must not race; use one grid per host thread.
 *   - Streams are the caller's (a hipStream_t passed as void*; NULL is the
 *     null stream).  Stepping is asynchronous on that stream.
 */
#ifndef RDMI_RD_H
#define RDMI_RD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RD_MAX_SPECIES 4
#define RD_ABI_VERSION 1

/* status codes */
enum {
    RD_OK = 0,
    RD_EINVAL = -1,      /* bad argument                                  */
    RD_ENOMEM = -2,      /* device allocation failed / over the HBM budget */
    RD_EUNSTABLE = -3,   /* dt outside the explicit scheme's stable range  */
    RD_ESTATE = -4,      /* call out of order (e.g. rd_step before model)  */
    RD_EDEVICE = -5,     /* HIP runtime or kernel error                    */
    RD_ENONFINITE = -6   /* a reduction found NaN or Inf in the field      */
};

/* element types of stored fields and of host/device transfers */
enum { RD_F32 = 0, RD_BF16 = 1, RD_F16 = 2, RD_F64 = 3 };

/* models (section 4.1 and Table 1 families) */
enum {
    RD_MODEL_DIFFUSION = 0,    /* R = 0; 1..4 independent species             */
    RD_MODEL_BRUSSELATOR = 1,  /* 2 species u, v: activator-inhibitor Turing   */
    RD_MODEL_FRONT_CH = 2,     /* 3 species A, B, C: front + Cahn-Hilliard     */
    RD_MODEL_POLLUTANT = 3,    /* 1..4 species: advection-diffusion + sources  */
    RD_MODEL_TURING = 4,       /* 2 species: Table 1's activator-inhibitor     */
    RD_MODEL_ATMOS = 5         /* 1..4 species: Table 1's atmospheric wind     */
};

/* boundary rule of one face of one species (section 4.1, Table 1) */
enum {
    RD_BC_MIRROR = 0,    /* no-flux / zero-gradient / outflow: ghost = edge cell */
    RD_BC_PERIODIC = 1,  /* ghost = cell at the other end (both faces of the axis) */
    RD_BC_GHOST = 2,     /* ghost = bc_value (e.g. clean inflow: 0)              */
    RD_BC_HELD = 3       /* the face's cell layer is held at bc_value, never
                            updated (Dirichlet layer).  A cell on several held
                            faces takes the first in the order x-,x+,y-,y+,z-,z+ */
};

/* faces, in this order everywhere */
enum { RD_FACE_XLO = 0, RD_FACE_XHI, RD_FACE_YLO, RD_FACE_YHI, RD_FACE_ZLO, RD_FACE_ZHI };

/*
 * rd_model_desc -- the whole definition of one explicit step.
 *
 * diff[s][d]   diffusion coefficient of species s along axis d (x, y, z), in
 *              length^2/time; isotropic D is diff[s][0..2] = D (Eq. (2)).
 * param[]      model constants:
 *   DIFFUSION    none
 *   BRUSSELATOR  [0]=a [1]=b      R_u = a-(b+1)u+u^2 v,  R_v = b u - u^2 v
 *   FRONT_CH     [0]=k [1]=M [2]=kappa [3]=eps [4]=gamma [5]=k2 (>= 0)
 *                r = k A B, q = k2 A C (redissolution);  R_A = -r - q,
 *                R_B = -r;  R_C = r - q + M Lap(mu),
 *                mu = gamma C^3 - eps C - kappa Lap(C)  (Table 1, third row,
 *                with lambda = M, sigma = kappa).  mu uses mirror ghosts on
 *                every face.  diff[2] may be 0 (C moves by the CH term only).
 *   POLLUTANT    [0]=lambda (first-order decay of every species)
 *                [1]=k_AB   (linear transfer species 0 -> species 1)
 *                A_s = -u(z) (c_s(i) - c_s(i-1)) / h, first-order upwind
 *                along +x with u(z) >= 0 (section 4.1, Table 1 fourth row)
 *   TURING       [0]=alpha [1]=beta [2]=gamma   (Table 1, second row)
 *                R_1 = c_1 - c_1^3 - c_2,  R_2 = gamma (c_1 - alpha c_2 - beta)
 *   ATMOS        [0]=u_x [1]=u_y [2]=u_z amplitude [3]=T (>= 0) [4]=t_0
 *                (Table 1, last row) a wind uniform in space, u_z(t) =
 *                u_z sin(t / T) (u_z itself when T = 0), t = t_0 + n dt at
 *                the n-th step since rd_set_model; every axis is upwinded
 *                by the sign of its component, A_s = sum_d of u_d (c[-e_d]
 *                - c) / h (u_d > 0) or u_d (c - c[+e_d]) / h (u_d < 0);
 *                species are independent; point sources as below.  The
 *                step index lives on the device, so graph replays see the
 *                time advance.  Not blocked in time (RD_KERNEL_LDS2) and not
 *                batched.
 * wind         POLLUTANT: nz host doubles u(z) >= 0, read during the call.
 * src_*        POLLUTANT, ATMOS: nsrc point sources, host arrays read during the
 *              call: linear cell index (k*ny + j)*nx + i, species, rate
 *              (added to dc/dt; duplicates add up).
 * stencil      7 (or 0): the 7-point Laplacian with per-axis coefficients;
 *              19: the 19-point Laplacian of Eqs. (3)-(4), weights -24 (centre),
 *              2 (faces), 1 (edges) over 6h^2, for isotropic diff[s][0..2]
 *              only (RD_EINVAL otherwise).  An edge neighbour outside two
 *              faces takes the rule of the first of them in x, y, z order.
 *              19-point grids run on the direct and LDS-ring plans and are
 *              not batched.
 * integrator   0 or RD_EULER: forward Euler, Eq. (5).  RD_RK2 / RD_RK3: the
 *              strong-stability-preserving Runge-Kutta steps of order 2
 *              (Heun) and 3 (Shu-Osher) built from Euler steps E(u) = u +
 *              dt F(u): RK2  c' = c + (E(E(c)) - c)/2;  RK3  u = c +
 *              (E(E(c)) - c)/4,  c' = c + 2 (E(u) - c)/3 (the paper notes
 *              that more accurate steppers exist, section 2).  Each Euler
 *              stage keeps held layers, and the combinations keep them
 *              exactly.  The combinations are fused into the stages' stores
 *              (each stored value v becomes c + w (v - c) at the same
 *              element).  An order-3 grid allocates one more buffer per
 *              species.  Runge-Kutta grids take no two-step plan
 *              (RD_KERNEL_LDS2), are not batched, and refuse the atmospheric
 *              model (its wind depends on time) with RD_EINVAL.
 * dt           time step; rd_set_model rejects a dt outside the stable range
 *              (RD_EUNSTABLE): per species dt*(2*sum_d K_d/h^2 + max u/h) <= 1
 *              (19-point: dt*(4 D/h^2 + max u/h) <= 1; for ATMOS, max u is
 *              |u_x| + |u_y| + |u_z|), and for FRONT_CH also
 *              dt*M*(kappa*L^2 + |eps|*L) <= 1 with L = 12/h^2 (19-point:
 *              16/(3h^2)), the largest magnitude of the discrete Laplacian.
 */
typedef struct rd_model_desc {
    int32_t model;
    int32_t nspecies;
    double dt;
    double diff[RD_MAX_SPECIES][3];
    int32_t bc_kind[RD_MAX_SPECIES][6];
    double bc_value[RD_MAX_SPECIES][6];
    double param[8];
    const double *wind;
    int64_t nwind;
    int64_t nsrc;
    const int64_t *src_cell;
    const int32_t *src_species;
    const double *src_rate;
    int32_t stencil;
    int32_t integrator;
} rd_model_desc;

/* time integrators (rd_model_desc.integrator) */
enum { RD_EULER = 1, RD_RK2 = 2, RD_RK3 = 3 };

/* kernel plan of a grid (all plans give bitwise-identical fields) */
enum {
    RD_KERNEL_AUTO = 0,    /* library choice: the rd_autotune cache entry for
                              this shape, model and integrator, else a heuristic
                              (the one-pass plan for the 7-point front model; a
                              slab shape for other 7-point models; for 19-point
                              ones the first LDS-ring shape, with z chunks for
                              about two workgroups per CU)                      */
    RD_KERNEL_DIRECT = 1,  /* one thread per cell, neighbours through the cache */
    RD_KERNEL_TILED = 2,   /* xy tile per workgroup, z-march register window,
                              wave64 lane shifts for x, LDS for inter-wave rows */
    RD_KERNEL_BLOCK = 3,   /* xy tile x cz-plane slab per workgroup, all planes
                              loaded up front; same lane shifts and LDS rows    */
    RD_KERNEL_LDS = 4,     /* FP32 or BF16 rows of up to 256 (vx 4) or 512 (vx 8)
                              cells, more than 256 for vx 8, nx a multiple of 4
                              (FP32) or 8 (BF16): z-march over a ring of LDS
                              plane slots filled by direct-to-LDS loads from one
                              producer wave                                    */
    RD_KERNEL_LDS2 = 5,    /* as RD_KERNEL_LDS, two time steps per launch
                              (temporal blocking; diffusion and Brusselator).
                              rd_step with an odd count finishes with one
                              direct-kernel step                               */
    RD_KERNEL_FUSED = 6,   /* FRONT_CH with the 7-point Laplacian only: the
                              whole step in one launch (the Cahn-Hilliard
                              chemical potential computed in LDS one plane
                              ahead of the update, no mu array in HBM; the two
                              Laplacian passes of section 4.1 fused).  128-cell
                              x tiles, any nx (a periodic x axis of C needs
                              nx <= 128 or a multiple of 128)                  */
    RD_KERNEL_TRING = 7    /* FP32 or BF16, 7-point diffusion of one or two
                              species, Brusselator and the pollutant's passes
                              of one or two species: z-march over
                              128-cell x tiles of ry rows, every field streamed
                              into an LDS ring by one loading wave, any nx     */
};
typedef struct rd_plan {
    int32_t kernel;       /* RD_KERNEL_*                                        */
    int32_t vx;           /* TILED/BLOCK: cells per lane along x (1, 2 or 4);
                             LDS: 4 (rows of <= 256 cells) or 8 (257..512);
                             LDS2: 4 (rows of 256 cells) or 8 (of 512);
                             FUSED: waves computing the chemical potential;
                             TRING: 2 (cells per lane)                         */
    int32_t ry;           /* TILED/BLOCK: rows per wave (1, 2 or 4);
                             LDS/LDS2/FUSED/TRING: rows per workgroup          */
    int32_t waves;        /* TILED/BLOCK: waves per workgroup (1 or 4);
                             LDS/LDS2: computing waves (plus one loading wave);
                             FUSED: waves updating the fields (plus vx waves
                             for the chemical potential and one loading wave);
                             TRING: computing waves (plus one loading wave, or
                             two when the fields' ring rows times prefetch-3
                             exceed 63 loads)                                  */
    int32_t cz;           /* TILED/LDS/LDS2/FUSED/TRING: z planes per workgroup, 0 = all;
                             BLOCK: planes per slab (2, 4 or 8)                */
    int32_t prefetch;     /* TILED: planes in flight ahead of the z window (1-2);
                             LDS/LDS2/FUSED/TRING: input ring slots            */
    int32_t order;        /* BLOCK/LDS/LDS2/FUSED/TRING: tile enumeration, 0 = x, then y, then z chunk;
                             1 = z chunk fastest (z-neighbour slabs run together
                             on one XCD and share its L2)                       */
    int32_t graph_chunk;  /* rd_step replays hipGraphs of this many steps (even,
                             >= 2); 0 launches every step directly            */
} rd_plan;

typedef struct rd_grid rd_grid;
typedef struct rd_batch rd_batch;

/* ----------------------------------------------------------------- grids */

/* Allocate a grid: two device buffers per species (the "first" and "second"
 * arrays of Table 3 line 1), zero-filled, on the current HIP device.
 * storage_dtype is RD_F32, RD_BF16 or RD_F16.  hip_stream is borrowed, not
 * owned.  On success *out owns the device memory until rd_destroy_grid. */
int rd_create_grid(int64_t nx, int64_t ny, int64_t nz, int32_t nspecies, double h,
                   int32_t storage_dtype, void *hip_stream, rd_grid **out);

/* Install the model (copied; host arrays are read during the call only).
 * Validates it against the grid, including the stability bound. */
int rd_set_model(rd_grid *g, const rd_model_desc *m);

/* Copy one species' field into the current state (Table 3 line 2).
 * src is dense [nz][ny][nx] of src_dtype (RD_F32/RD_F64/RD_BF16/RD_F16),
 * on the host (src_on_device = 0) or the device (1 or 2); values are
 * converted to the storage type with round-to-nearest-even.  0 and 1 are
 * synchronous.  2 only enqueues the copy on the grid's stream and returns:
 * the caller keeps src alive and unchanged until the stream has passed that
 * point, and must have ordered src's own producer before it (for a serving
 * loop that builds initial states on the grid's stream while earlier steps
 * still run).  Errors of an enqueued copy surface at the next synchronizing
 * call. */
int rd_write_field(rd_grid *g, int32_t species, const void *src, int32_t src_dtype,
                   int32_t src_on_device);

/* Advance n >= 0 explicit Euler steps (Table 3 lines 3-10), asynchronously on
 * the grid's stream. */
int rd_step(rd_grid *g, int64_t n);

/* Copy one species' current field out (Table 3 line 11), converting to
 * dst_dtype (RD_F32 or RD_F64 on the host; RD_F32 on the device).
 * Synchronises the grid's stream. */
int rd_read_field(rd_grid *g, int32_t species, void *dst, int32_t dst_dtype,
                  int32_t dst_on_device);

/* FP64 mass sum(c) h^3 and energy sum(c^2) h^3 of one species, reduced on the
 * GPU in a fixed order (deterministic).  Synchronises; RD_ENONFINITE if the
 * field holds NaN or Inf (out is still written). */
int rd_reduce(rd_grid *g, int32_t species, double out_mass_energy[2]);

/* FRONT_CH only: the Cahn-Hilliard chemical potential mu of the current state
 * (FP32, the first of the two Laplacian passes; with the one-pass plan the
 * direct kernel computes it), dense [nz][ny][nx] on the host.  Synchronises. */
int rd_chemical_potential(rd_grid *g, float *dst_host);

/* Allocation-free reduction, for callers that cannot allocate device memory
 * (code under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the FP64 mass sum(c) h^3 and energy sum(c^2) h^3 of a dense
 * [nz][ny][nx] device field of dtype RD_F32, RD_BF16 or RD_F16 at `field`,
 * written to out_dev[0], out_dev[1] (caller-owned device memory), with the
 * same kernels and summation order as rd_reduce (so a grid's field and a
 * dense copy of it give the same bits).  Asynchronous on hip_stream; nothing
 * is allocated and nothing synchronised.  The partial sums live in a fixed
 * 16 KiB per-GPU array inside the library (2 x 1024 doubles, held until the
 * process ends), so calls that overlap on one GPU race and must be ordered by
 * the caller (one stream, or events).  Fields up to the largest grid
 * (extents <= 2^24, 2^40 cells) are accepted, RD_EINVAL beyond; non-finite
 * values give non-finite results (no check, no synchronisation). */
int rd_reduce_noalloc(const void *field, int32_t dtype, int64_t nx, int64_t ny, int64_t nz, double h,
                      double *out_dev, void *hip_stream);

/* Wait for the grid's stream; RD_EDEVICE if a kernel failed. */
int rd_sync(rd_grid *g);

int rd_destroy_grid(rd_grid *g);

/* Device bytes rd_create_grid would allocate for this shape (both time
 * levels, padding and the Cahn-Hilliard work field when with_aux != 0).
 * Pure host computation, usable for admission control. */
size_t rd_grid_bytes(int64_t nx, int64_t ny, int64_t nz, int32_t nspecies,
                     int32_t storage_dtype, int32_t with_aux);

/* Host-only validation of a model for a grid shape (what rd_set_model
 * checks before touching the device). */
int rd_validate_model(int64_t nx, int64_t ny, int64_t nz, int32_t nspecies, double h,
                      const rd_model_desc *m);

/* ----------------------------------------------------------------- plans */

int rd_set_plan(rd_grid *g, const rd_plan *p);   /* RD_EINVAL if unsupported */
int rd_get_plan(const rd_grid *g, rd_plan *p);   /* the plan rd_step uses    */

/* Kernel launches per Euler step (per Runge-Kutta stage) of the grid's model
 * (*out): 1, or 2 for the front model (chemical-potential pass, then the
 * update; 1 with RD_KERNEL_FUSED) and for more than two species of the pollutant and atmospheric
 * models (species groups that share no term, section 2's Eq. (5) evaluated
 * group by group).  RD_ESTATE without a model. */
int rd_get_passes(const rd_grid *g, int32_t *out);

/* rounding of stored BF16 values (rd_set_rounding) */
enum { RD_ROUND_NEAREST = 0, RD_ROUND_STOCHASTIC = 1 };

/* How a step rounds the values it stores into BF16 fields (the arithmetic
 * stays FP32).  RD_ROUND_NEAREST (the default): round to nearest even.
 * RD_ROUND_STOCHASTIC: round the magnitude up with probability (discarded low
 * 16 bits) / 2^16, so the expected stored value is the FP32 result and
 * increments smaller than half a BF16 unit do not stagnate.  The random bits
 * are Philox-2x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): element e of a
 * field (its dense index (z*ny + y)*nx + x) takes 16 of the 64 output bits of
 * counter (e/4 mod 2^32, step index since rd_set_model) and key (low 32 bits
 * of seed + species) -- bits 0-15 of the first output word for e%4 = 0, bits
 * 16-31 for 1, the same halves of the second word for 2 and 3 -- so one call
 * serves four elements.  The same inputs give the same bits on every plan, in
 * graphs and whatever the internal padding (fields of up to 2^34 elements
 * have distinct counters).  Kept across rd_set_model.  RD_EINVAL:
 * unknown mode, or stochastic rounding with storage other than RD_BF16 or a
 * Runge-Kutta model; RD_ESTATE: the grid is in a batch (batches refuse
 * grids with stochastic rounding). */
int rd_set_rounding(rd_grid *g, int32_t mode, uint64_t seed);

/* Time candidate plans on this grid (trial_steps steps each, hipEvents on the
 * grid's stream), keep the fastest, store it in a per-process cache keyed by
 * shape, species, model and storage, and return it in *best.  The grid's state
 * is saved before and restored after, so the call leaves the fields as they
 * were.  Synchronous. */
int rd_autotune(rd_grid *g, int32_t trial_steps, rd_plan *best);

/* ---------------------------------------------------------- batched form */

/* A batch steps many grids of uneven size together: each launch is one
 * persistent kernel that walks a work list of (grid, tile) items covering
 * every active grid, and rd_batch_step replays a captured hipGraph of such
 * launches.  Grids must use the DIFFUSION or BRUSSELATOR model, share the
 * batch's storage dtype and stay alive while in the batch.
 * hbm_budget_bytes caps the summed rd_grid_bytes of member grids. */
int rd_batch_create(int32_t max_grids, size_t hbm_budget_bytes, int32_t storage_dtype,
                    void *hip_stream, rd_batch **out);

/* Add a grid with `steps` steps to run.  RD_ENOMEM if it would exceed the HBM
 * budget, RD_EINVAL if the batch is full or the grid is unsuitable.  The
 * grid's own stream is synchronised first. */
int rd_batch_add(rd_batch *b, rd_grid *g, int64_t steps);

/* Run up to `chunk` steps of every member (members with fewer steps left stop
 * early), asynchronously on the batch stream.  Writes to finished[] (capacity
 * max_grids) the grids whose steps are all done once this chunk completes and
 * removes them from the batch; *n_finished is their count. */
int rd_batch_step(rd_batch *b, int64_t chunk, rd_grid **finished, int32_t *n_finished);

/* Remove a grid before it finished (its state is left as stepped so far). */
int rd_batch_remove(rd_batch *b, rd_grid *g);

/* Members, bytes in use, steps still to run summed over members. */
int rd_batch_info(const rd_batch *b, int32_t *n_members, size_t *bytes_in_use,
                  int64_t *steps_left_total);

int rd_batch_destroy(rd_batch *b);

/* ----------------------------------------------------------- measurement */

/* Plain device-to-device copy kernel of `bytes` (a multiple of 16) on the
 * given stream: the bandwidth ceiling a read+write stream can reach. */
int rd_copy_probe(void *dst, const void *src, size_t bytes, void *hip_stream);

const char *rd_last_error(void);
int rd_abi_version(void);

/* Digest of the kernel and engine sources this library was built from (16
 * hex digits of a SHA-256 over csrc/, computed by the build and compiled in;
 * "unknown" if built without it).  Static string, never NULL.  Lets a caller
 * check that the binary it loaded matches the sources it ships with. */
const char *rd_source_digest(void);

#ifdef __cplusplus
}
#endif
#endif /* RDMI_RD_H */
