/*
 * glbm: Gaussian lattice Boltzmann hierarchy on MI355X (gfx950).
 *
 * C-ABI of the HIP library libglbm.so.  The library advances the models of
 * O. Ilyin, "Gaussian Lattice Boltzmann method and its applications to
 * rarefied flows" (arXiv:1905.04597): the G-D1Q(2N+1) models of section 2
 * (update Eq. maineq01, equilibrium Eqs. maineq02-maineq06 = the N-fold
 * convolution of the D1Q3 equilibrium at velocity u/N) and their tensor
 * products in two dimensions (section 4), with the linear body force of
 * section 5.4, diffuse-reflection walls (sections 5.3, 5.4) and fixed
 * equilibrium ends (section 5.1).
 *
 * Units are lattice units: time step 1 and lattice spacing 1 on each axis,
 * so a level-N axis has velocities -N..N and temperature theta = N/3
 * (Eq. maineq05 with c = 1).  Velocities are reported in these units.
 *
 * Conventions shared by every entry point:
 *  - Velocity index q = b * (2 Nx + 1) + a for the velocity (a - Nx, b - Ny),
 *    Nx, Ny the levels of the two axes (one dimension: Ny = 0, q = a).
 *  - Canonical arrays (fields and FP32 populations exchanged with the
 *    caller) are row-major [y][x] per field and [q][y][x] for populations,
 *    x fastest, no padding.
 *  - All pointers passed to the library are DEVICE pointers on the device
 *    that was current when glbm_create was called, unless stated otherwise.
 *    The caller owns them (PyTorch allocations in the Python binding) and
 *    keeps them alive while the handle uses them.
 *  - Work is enqueued on the caller's HIP stream, asynchronously, unless an
 *    entry point says that it synchronizes.
 *  - Every call returns GLBM_OK (0) or a negative error code; the message of
 *    the last failure on the calling thread is glbm_last_error().  No C++
 *    exception crosses this interface.
 *
 * Time convention: after glbm_init_* the solver is at time t = 0 with
 * pre-collision populations f(0); each glbm_step advances t by one
 * (collision, then streaming, Eq. maineq01).  glbm_moments and
 * glbm_get_populations report the pre-collision state f(t).
 */
#ifndef GLBM_H
#define GLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define GLBM_OK 0
#define GLBM_ERR_INVALID (-1)     /* invalid argument or configuration */
#define GLBM_ERR_UNSUPPORTED (-2) /* valid but not built (level, storage, boundary combination) */
#define GLBM_ERR_HIP (-3)         /* a HIP runtime call failed */
#define GLBM_ERR_STATE (-4)       /* call out of order (e.g. step before init) */
#define GLBM_ERR_NONFINITE (-5)   /* glbm_stats: some node's density, momentum or energy is not a
                                     finite number (the run has blown up) */
#define GLBM_ERR_POSITIVITY (-6)  /* glbm_stats: some node's velocity is outside the domain in
                                     which the equilibrium is non-negative (section 3) */

/* Boundary kinds. */
#define GLBM_BC_PERIODIC 0
#define GLBM_BC_WALL 1    /* diffuse-reflection wall (y axis, two dimensions) */
#define GLBM_BC_EQ_ENDS 2 /* fixed equilibrium ends at rest (x axis) */

/* Population storage. */
#define GLBM_STORE_F32 0          /* f in FP32 */
#define GLBM_STORE_F32_SHIFTED 1  /* f - S in FP32: S is the rest state W_a W_b rounded to
                                     multiples of 2^-24 with unit sum (deviation storage); the
                                     relaxation update is rounded without bias (dithered by
                                     one unit in the last place, random bits keyed by (time
                                     step, node, velocity): reproducible) */
#define GLBM_STORE_BF16_SHIFTED 2 /* f - S in BF16, round to nearest even.  Undriven lattices
                                     only (no force, no walls): per-step increments below half
                                     a BF16 unit are lost, so a driven flow stalls; creation
                                     with a force or walls returns GLBM_ERR_UNSUPPORTED */
#define GLBM_STORE_BF16_SHIFTED_SR 3 /* f - S in BF16, stochastic rounding keyed by
                                        (time step, node, velocity): reproducible */

/* Largest hierarchy level per axis built into the library: 7 on every axis,
 * and 13 for the G-D1Q(2N+2) axis across the walls of the mixed channel
 * lattices D1Q3 x G-D1Q(2N+2) (the paper's G-D1Q20 ... G-D1Q28 x D1Q3 of
 * section 5.4).  Levels 8..13 elsewhere pass the configuration checks but
 * glbm_create returns GLBM_ERR_UNSUPPORTED. */
#define GLBM_MAX_LEVEL 13
#define GLBM_MAX_LEVEL_ANY_AXIS 7

/* Velocity set of an axis (section 2). */
#define GLBM_AXIS_ODD 0  /* G-D1Q(2N+1): velocities -N..N, theta = N/3 (unit lattice step) */
#define GLBM_AXIS_EVEN 1 /* G-D1Q(2N+2), zero velocity removed (Eqs. maineq01_noball-
                            maineq04_noball): velocities (n + 1/2) c on a grid of half the
                            lattice step c, i.e. the odd integers -(2N+1)..2N+1 in grid
                            units, theta = (4N+3)/3 (Eq. temp_2N2 with c = 2 grid units).
                            Built: one dimension (N = 1..7), the mixed lattices
                            G-D1Q3 x G-D1Q(2N+2) with walls across the even axis (the form of
                            sections 5.3-5.4, N = 1..13) and the symmetric two-dimensional
                            products (N = 1..7). */

typedef struct glbm_config {
    int32_t dims;     /* 1, 2 or 3 */
    int32_t level_x;  /* hierarchy level N of the x axis, 1..GLBM_MAX_LEVEL */
    int32_t level_y;  /* level of the y axis (two dimensions), 1..GLBM_MAX_LEVEL; ignored in 1D */
    int32_t storage;  /* GLBM_STORE_* */
    int64_t nx, ny;   /* nodes per axis; ny is ignored (1) in one dimension */
    double tau;       /* relaxation time (> 0), or <= 0 to derive it from kn */
    double kn;        /* Knudsen number of Eq. kn: tau = kn H / sqrt(2 theta), with
                         H = ny and theta of the y axis in two dimensions (walls half
                         way between nodes), H = nx and theta of the x axis in one */
    int32_t bc_x;     /* GLBM_BC_PERIODIC or GLBM_BC_EQ_ENDS */
    int32_t bc_y;     /* GLBM_BC_PERIODIC or GLBM_BC_WALL (two dimensions) */
    double wall_u[2]; /* x velocity of the bottom (y = -1/2) and top (y = ny - 1/2) walls */
    double end_rho[2];/* densities of the left (x < 0) and right (x >= nx) equilibrium ends */
    double g;         /* body force along x: momentum added per node and step */
    int32_t kind_x;   /* GLBM_AXIS_ODD or GLBM_AXIS_EVEN */
    int32_t kind_y;   /* GLBM_AXIS_ODD or GLBM_AXIS_EVEN (two dimensions); ignored in 1D */
    /* Three dimensions (dims = 3): the tensor product of three axes (section 4
     * with a third factor), periodic in x and z, periodic or walls in y.
     * Built: D3Q27 (levels 1,1,1), G-D3Q125 (2,2,2), G-D3Q343 (3,3,3),
     * D1Q3 x G-D1Q(2N+1) x D1Q3 (1,N,1, N = 2..7) and D1Q3 x G-D1Q(2N+2) x D1Q3
     * (1,N,1 with kind_y EVEN, N = 2..7).  Batches take every one of them but
     * G-D3Q343.  Ignored in one and two dimensions. */
    int64_t nz;       /* nodes along z (>= the fastest z velocity) */
    int32_t level_z;  /* level of the z axis, 1..GLBM_MAX_LEVEL */
    int32_t kind_z;   /* GLBM_AXIS_ODD or GLBM_AXIS_EVEN */
} glbm_config;

/* Global diagnostics, FP64 sums over all nodes (glbm_stats). */
typedef struct glbm_stats {
    int64_t time;           /* t */
    double mass;            /* sum of f(t) */
    double momentum_x;      /* sum of f(t) c_x (pre-collision) */
    double momentum_y;      /* sum of f(t) c_y */
    double energy_post;     /* sum of f*(t) |c|^2 after the collision of step t (the model
                               is isothermal: reported, not conserved) */
    double residual;        /* ||u_x(t) - u_x(t-1)||_2 / ||u_x(t)||_2; NaN at t = 0 */
    double wall_mass[2];    /* mass absorbed (and re-emitted) by the bottom/top wall in the
                               streaming from t to t+1 */
    double wall_momentum[2];/* x momentum given to the bottom/top wall in that streaming */
    double nonpositive_nodes; /* nodes with u^2 above 2 N theta0 on some axis (theta0 of the
                                 underlying 2N+1 walk: N/3, or 4N/3 on an even axis's half grid)
                                 (equilibrium not positive, section 3) */
    double momentum_z;      /* sum of f(t) c_z (three dimensions; 0 otherwise) */
    double nonfinite_nodes; /* nodes whose density, momentum or energy is not a finite number
                               (not counted in nonpositive_nodes; they make the sums above
                               non-finite) */
} glbm_stats_t;

typedef struct glbm_solver glbm_t;

/* Bytes of ONE population buffer for cfg (the library's internal layout:
 * velocity planes [q][row][column], each plane rounded up to 256 bytes; two-
 * and three-dimensional lattices have compact rows of exactly nx columns
 * (rows y, or z * ny + y), one-dimensional ones one row of nx columns plus
 * ghost columns padded to a multiple of 64), or 0 if cfg is invalid.  The caller
 * allocates two such buffers on the device (for HBM-budget admission this is
 * the whole device footprint apart from a few KB of tables). */
size_t glbm_population_bytes(const glbm_config *cfg);

/* Device bytes a solver of cfg occupies in total: its two population buffers
 * (caller-owned), the FP64 statistics buffers the library allocates on the
 * first glbm_stats call (a fixed number of partial-sum rows, at most
 * 2048 x 13 doubles) and, for the lattices with walls whose step starts
 * with a wall pre-pass (three dimensions; the symmetric G-D1Q(2N+2) products
 * at N = 6, 7), the per-column wall factors the library allocates at
 * glbm_create (2 nx nz floats, nz = 1 in two dimensions); 0 if cfg is
 * invalid.  For HBM-budget admission. */
size_t glbm_required_bytes(const glbm_config *cfg);

/* Create a solver over caller-owned device buffers pop_a and pop_b, each of
 * glbm_population_bytes(cfg) bytes, 256-byte aligned, on HIP stream `stream`
 * (hipStream_t; NULL = the default stream).  The relaxation time is cfg->tau,
 * or, with tau <= 0, the one Eq. kn gives for cfg->kn (kinematic viscosity
 * nu = theta tau, section 5.2: tau = Kn H / sqrt(2 theta)); the collision
 * frequency of Eq. maineq01 is 1 / (tau + 1/2).  The state is undefined until
 * glbm_init_fields or glbm_init_populations.  *out receives the handle; the
 * caller keeps the buffers alive until glbm_destroy.  The lattices whose
 * step takes a wall pre-pass allocate their wall factors here (see
 * glbm_required_bytes); nothing else is allocated before glbm_stats.
 * Errors: GLBM_ERR_INVALID for a bad configuration (including omega outside
 * (0, 2), ny < 2 Ny with walls, walls combined with equilibrium ends, a
 * buffer above 4 GiB), GLBM_ERR_UNSUPPORTED for level combinations not built
 * and for round-to-nearest BF16 storage with a force or walls. */
int glbm_create(const glbm_config *cfg, void *pop_a, void *pop_b, void *stream, glbm_t **out);

/* f(0) = f^eq(rho, u) at every node (Eqs. maineq02-maineq06 per axis, product
 * form of section 4).  rho, ux, uy: device float arrays [ny][nx]; NULL means
 * rho = 1, u = 0.  Sets t = 0. */
int glbm_init_fields(glbm_t *h, const float *rho, const float *ux, const float *uy);

/* f(0) given: device float array [Q][ny][nx] of pre-collision populations.
 * Sets t = 0. */
int glbm_init_populations(glbm_t *h, const float *f0);

/* Advance nsteps >= 0 time steps (each: moments, equilibrium, BGK collision
 * with force, wall densities, pull streaming; one fused kernel per step). */
int glbm_step(glbm_t *h, int64_t nsteps);

/* Moments of f(t) (the hydrodynamic moments of section 2: density sum f,
 * momentum sum f c, and the second moments): density, velocity u = sum f c /
 * rho, temperature per degree of freedom T = (sum f |c|^2 / rho - |u|^2) /
 * dims and shear moment Pxy = sum f c_x c_y - rho u_x u_y, summed in FP64 and
 * rounded to FP32.  Device float arrays [ny][nx]; any may be NULL (skipped).
 * Asynchronous on the solver's stream. */
int glbm_moments(glbm_t *h, float *rho, float *ux, float *uy, float *T, float *pxy);

/* As glbm_init_fields, with the z velocity uz (three dimensions; may be NULL).
 * Fields are [nz][ny][nx]. */
int glbm_init_fields3(glbm_t *h, const float *rho, const float *ux, const float *uy, const float *uz);

/* As glbm_moments, with the z velocity uz (written in three dimensions only;
 * the temperature is then per degree of freedom over three axes).  Fields are
 * [nz][ny][nx]; any pointer may be NULL. */
int glbm_moments3(glbm_t *h, float *rho, float *ux, float *uy, float *uz, float *T, float *pxy);

/* Copy f(t) (pre-collision, FP32, canonical [Q][nz][ny][nx], q = (c Qy + b) Qx
 * + a) into device memory. */
int glbm_get_populations(glbm_t *h, float *out);

/* Global FP64 diagnostics at the current time.  Synchronizes the stream.  The
 * first call allocates the solver's small FP64 reduction buffers.  *out is
 * filled in every case where the sums were read; the status then reports the
 * state's health: GLBM_ERR_NONFINITE if some node is not finite (the run has
 * blown up), else GLBM_ERR_POSITIVITY if some node's velocity is outside the
 * positivity domain of section 3 (|u| <= sqrt(2 N theta0) per axis), else
 * GLBM_OK. */
int glbm_stats(glbm_t *h, glbm_stats_t *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): as
 * glbm_stats, but the FP64 partial sums go through a fixed device array of
 * the library (2049 x 13 doubles, 213 KB, held once per GPU until the process
 * ends) instead of buffers allocated on the first call; it allocates nothing.
 * Any lattice the library accepts fits (the statistics blocks stride over the
 * nodes; a larger need would return GLBM_ERR_INVALID).  Every call on one GPU
 * shares that array: calls that overlap on one GPU (other host threads, other
 * streams) race and must be serialised by the caller.  Same statuses as
 * glbm_stats. */
int glbm_stats_static(glbm_t *h, glbm_stats_t *out);

/* Derived parameters: relaxation time, collision frequency 1/(tau + 1/2),
 * number of velocities, current time.  Host pointers; any may be NULL. */
int glbm_info(const glbm_t *h, double *tau, double *omega, int32_t *nvel, int64_t *time);

/* Release the handle (host state, and the FP64 reduction buffers if
 * glbm_stats allocated them: then it first waits for the handle's stream).
 * Caller-owned buffers are not touched: keep them until the work enqueued on
 * them has run. */
int glbm_destroy(glbm_t *h);

/* Message of the last failing call on this thread ("" if none). */
const char *glbm_last_error(void);

/* ------------------------------------------------------------------------
 * Batched stepping: many solvers advanced together (uneven sizes, levels,
 * dimensions and parameters).  Members of the same kernel variant (levels, storage,
 * boundaries) share one launch per step over a table of tiles, each tile a
 * run of nodes of one member; a chunk of steps is captured once into a HIP
 * graph and replayed.  Every node runs exactly the code of glbm_step, so a
 * member's populations are bitwise those of the member stepped alone
 * (stochastic-rounding seeds included).  The batch's device tables (a few
 * hundred bytes per member and per tile) are one allocation of the library,
 * uploaded from a pinned host copy.
 * ------------------------------------------------------------------------ */
#define GLBM_ORDER_MEMBER 0        /* tiles of each member contiguous */
#define GLBM_ORDER_INTERLEAVE 1    /* tiles dealt round-robin over the members */
#define GLBM_ORDER_LARGEST_FIRST 2 /* members by decreasing work, contiguous */

typedef struct glbm_batch_options {
    int32_t tile_nodes;  /* nodes per workgroup: 64, 128 or 256 (0 = 256) */
    int32_t order;       /* GLBM_ORDER_* */
    int32_t graph_steps; /* steps per captured HIP graph; 0 = plain launches */
    int32_t resident_nodes; /* one- and two-dimensional members of at most this many
                               nodes are stepped by one workgroup each, all steps of a
                               chunk in one launch per variant (small lattices: no
                               launch per step); 0 = none.  Three-dimensional members
                               are always tiled. */
    int32_t streams;     /* kernel variants advance side by side on up to this many
                            streams (1..8; 0 = 1): the batch's stream and streams - 1
                            more that the batch creates (default priority), joined
                            back into the batch's stream after every chunk; the
                            launches of one variant stay in order on one stream */
} glbm_batch_options;

typedef struct glbm_batch glbm_batch_t;

/* Group n >= 1 initialised solvers (host array of handles, each at most once,
 * all on the current device) into a batch that launches on `stream` (NULL =
 * the default stream, joined through events).  While a solver belongs to a
 * batch, glbm_step on it returns GLBM_ERR_STATE; glbm_moments, glbm_stats and
 * glbm_get_populations keep working (on the solver's own stream: synchronise
 * the two streams if they differ).  opt may be NULL (defaults).  The tables
 * are allocated here and released by glbm_batch_destroy. */
int glbm_batch_create(glbm_t *const *members, int32_t n, const glbm_batch_options *opt, void *stream,
                      glbm_batch_t **out);

/* Advance every member by nsteps >= 0 steps. */
int glbm_batch_step(glbm_batch_t *b, int64_t nsteps);

/* Replace the member set (continuous batching: solvers join and leave between
 * steps).  Same rules as glbm_batch_create, except that n may be 0 (an empty
 * batch steps as a no-op and keeps its tables); members of this batch may stay,
 * members left out are released (they may be stepped alone again once the
 * batch's stream has run the work enqueued so far).  The tables are
 * re-planned in place and uploaded on the batch's stream, so work already
 * enqueued runs with the old plan; device memory is allocated only when the
 * new plan is larger than any before.  On failure the old members stay in the
 * batch but it cannot step until an update succeeds. */
int glbm_batch_update(glbm_batch_t *b, glbm_t *const *members, int32_t n);

/* Release the batch (members stay valid and can be stepped alone again).
 * Waits for the batch's work. */
int glbm_batch_destroy(glbm_batch_t *b);

/* ------------------------------------------------------------------------
 * Measurement utility (not part of the method): the HBM rates of plain
 * streaming kernels on this GPU, the ceiling against which the step kernels'
 * bandwidth fractions are read, and a kernel of known byte count for
 * calibrating memory counters.  mode 0 copies `bytes` from src to dst, mode 1
 * reads src (dst: a 4-byte device word that is almost never written), mode 2
 * writes dst; 16-byte non-temporal accesses in grid-stride loops over
 * `blocks` workgroups of 256 lanes, enqueued on `stream`.  bytes must be a
 * positive multiple of 16 and the buffers 16-byte aligned device memory of
 * the caller; GLBM_ERR_INVALID otherwise. */
int glbm_bandwidth_probe(int32_t mode, const void *src, void *dst, size_t bytes, int32_t blocks, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GLBM_H */
