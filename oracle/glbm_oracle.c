/*
 * Reference oracle for the Gaussian lattice Boltzmann hierarchy
 * (O. Ilyin, "Gaussian Lattice Boltzmann method and its applications to
 * rarefied flows", arXiv:1905.04597).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, FP64 CPU
 * implementation that the tests, the smoke check and the CPU-baseline leg
 * of the benchmark compare the HIP library against.  The product path never
 * calls it, and it shares no code, header, table or helper with the HIP
 * library: every formula below is written out again from the paper.
 *
 * Units: lattice units, time step 1, lattice spacing c = 1 on every axis, so
 * a population with velocity index n moves n nodes per step.  With c = 1,
 * Eq. maineq05 fixes the temperature of a level-N axis at theta = N/3.
 * The paper's own setting (theta0 = 1, c(N) = sqrt(3/N), Eq. maineq06) is the
 * same model rescaled; orc_equilibrium_1d takes c and theta0 explicitly so
 * that it can also be evaluated in those units.
 *
 * Two kinds of axis (section 2):
 *   ORC_AXIS_ODD  - G-D1Q(2N+1): velocities n = -N..N (index a = n + N),
 *                   theta = N/3;
 *   ORC_AXIS_EVEN - G-D1Q(2N+2), zero velocity removed
 *                   (Eqs. maineq01_noball-maineq04_noball): velocities
 *                   (n + 1/2) c of the lattice step c, here on a grid of half
 *                   that step (c = 2 nodes), i.e. the odd integers
 *                   v = 2a - (2N+1), a = 0..2N+1; by Eq. temp_2N2 the
 *                   temperature is theta = (4N+3) c^2 / 12 = (4N+3)/3.
 * Velocity ordering and state layout (shared by every array here):
 *   axis x has Qx velocities cx[a], axis y Qy velocities cy[b], axis z Qz
 *   velocities cz[c] (a single velocity 0 on an absent axis);
 *   q = (c * Qy + b) * Qx + a;  arrays are [q][z][y][x], x fastest.
 *   Three dimensions (section 4: the tensor product of three axes) are
 *   periodic in z.
 *
 * Parity status of each function is stated in its comment; every one of
 * them is pinned by a CPU test (closed forms, worked example of Appendix A,
 * brute-force enumeration, an independent push-form stepper, invariants).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_BC_PERIODIC 0
#define ORC_BC_WALL 1     /* diffuse-reflection wall (only on y) */
#define ORC_BC_EQ_ENDS 2  /* fixed equilibrium ends (only on x) */
#define ORC_AXIS_ODD 0
#define ORC_AXIS_EVEN 1

/* ------------------------------------------------------------------ */
/* Equilibrium of one axis: section 2, Eqs. maineq02-maineq04 and the   */
/* negative-n rule that follows Eq. maineq06.                           */
/* ------------------------------------------------------------------ */

static double fact(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= (double)i;
    return r;
}

/* Probability that the sum of N i.i.d. three-outcome steps equals n c,
 * for n = -N..N (out[n+N]), times rho = 1.  Closed form Eq. maineq03 with
 * the step probabilities of Eq. maineq04 (temperature theta0 = c_s^2).
 * For n < 0 the same sum is taken with |n| and P+ and P- exchanged.
 * N = 0 is the trivial one-velocity axis (out[0] = 1). */
void orc_equilibrium_1d(int N, double c, double theta0, double u, double *out)
{
    if (N == 0) {
        out[0] = 1.0;
        return;
    }
    const double Pp = (theta0 + c * u + u * u / N) / (2.0 * c * c * N);
    const double Pm = (theta0 - c * u + u * u / N) / (2.0 * c * c * N);
    const double P0 = 1.0 - Pp - Pm;
    for (int n = -N; n <= N; ++n) {
        const int an = n < 0 ? -n : n;
        const double pp = n >= 0 ? Pp : Pm; /* the step towards sign(n) */
        const double pm = n >= 0 ? Pm : Pp; /* the step away from it   */
        double sum = 0.0;
        for (int m = 0; m <= (N - an) / 2; ++m) {
            const double ways = fact(N) / (fact(an + m) * fact(m) * fact(N - an - 2 * m));
            sum += ways * pow(pp, an + m) * pow(pm, m) * pow(P0, N - an - 2 * m);
        }
        out[n + N] = sum;
    }
}

/* The three step probabilities (P-, P0, P+) of Eq. maineq04. */
void orc_step_probabilities(int N, double c, double theta0, double u, double *out3)
{
    out3[2] = (theta0 + c * u + u * u / N) / (2.0 * c * c * N);
    out3[0] = (theta0 - c * u + u * u / N) / (2.0 * c * c * N);
    out3[1] = 1.0 - out3[0] - out3[2];
}

/* Equilibrium at rho = 1 of one axis in lattice units (unit grid spacing).
 * ODD: Eq. maineq03 with c = 1, theta0 = N/3.  EVEN: the 2N+1 equilibrium on
 * the lattice of step c = 2 (theta0 = N c^2 / 3), each velocity (n + 1/2) c
 * taking the average of the states at its two neighbours n c and (n + 1) c
 * (Eqs. maineq01_noball-maineq04_noball; the outermost ones have a single
 * neighbour).  out has 2N+1 (ODD) or 2N+2 (EVEN) entries. */
void orc_axis_equilibrium(int kind, int N, double u, double *out)
{
    if (kind == ORC_AXIS_ODD) {
        orc_equilibrium_1d(N, 1.0, N / 3.0, u, out);
        return;
    }
    double F[64];
    orc_equilibrium_1d(N, 2.0, 4.0 * N / 3.0, u, F);
    for (int a = 0; a <= 2 * N + 1; ++a) {
        const double lo = a >= 1 ? F[a - 1] : 0.0;    /* neighbour n c, n = a - N - 1 */
        const double hi = a <= 2 * N ? F[a] : 0.0;     /* neighbour (n + 1) c */
        out[a] = 0.5 * (lo + hi);
    }
}

/* Relaxation time from the Knudsen number of Eq. kn (section 5.2):
 * Kn = sqrt(2/theta) nu / H with nu = theta tau, hence
 * tau = Kn H / sqrt(2 theta). */
double orc_tau_from_kn(double kn, double H, double theta)
{
    return kn * H / sqrt(2.0 * theta);
}

/* ------------------------------------------------------------------ */
/* Solver                                                               */
/* ------------------------------------------------------------------ */

typedef struct orc_solver {
    int dims, Lx, Ly, Lz;
    int kx, ky, kz;   /* axis kinds (ORC_AXIS_*) */
    int cx[64], cy[64], cz[64]; /* velocities of the three axes */
    double u2x, u2y, u2z; /* positivity bounds on u^2 of the axes (section 3) */
    int64_t nx, ny, nz;
    double tau, omega, g;
    int bc_x, bc_y;
    double wall_u[2]; /* x velocity of the bottom (y = -1/2) and top (y = ny - 1/2) wall */
    double end_rho[2];/* densities of the fixed equilibrium ends (x < 0, x >= nx) */
    int Qx, Qy, Qz, Q;
    double thx, thy, thz; /* axis temperatures in lattice units */
    double *Wx, *Wy, *Wz; /* rest weights: equilibrium at rho = 1, u = 0 */
    double Jplus_y;   /* half flux sum_{n>0} n W_n of the wall-normal axis */
    double *Ebot, *Etop; /* wall emission per velocity at unit wall density */
    double *f;        /* pre-collision populations f(t) */
    double *fs;       /* post-collision populations f*(t) (scratch) */
    double *fn;       /* next pre-collision state (scratch) */
    double *ux_prev;  /* u_x(t-1) per node, for the steady-state residual */
    double *rw_bot, *rw_top; /* wall densities per (x, z) column (scratch) */
    int64_t t;
} orc_solver;

static int64_t imod(int64_t a, int64_t m)
{
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

static inline int64_t nodes(const orc_solver *s) { return s->nx * s->ny * s->nz; }

/* Velocities, temperature and positivity bound of an axis.  Positivity
 * (section 3): P0 >= 0 of the underlying 2N+1 model, u^2 <= 2 N theta0 with
 * theta0 = N c^2 / 3 of its lattice step c (1 for ODD, 2 for EVEN). */
static int axis_setup(int kind, int N, int *vel, double *theta, double *u2max)
{
    if (kind == ORC_AXIS_ODD) {
        for (int a = 0; a <= 2 * N; ++a) vel[a] = a - N;
        *theta = N / 3.0;
        *u2max = 2.0 * N * (N / 3.0);
        return 2 * N + 1;
    }
    for (int a = 0; a <= 2 * N + 1; ++a) vel[a] = 2 * a - (2 * N + 1);
    *theta = (4.0 * N + 3.0) / 3.0;
    *u2max = 2.0 * N * (4.0 * N / 3.0);
    return 2 * N + 2;
}

/* Create a solver.  Returns NULL on an invalid configuration.
 * kind_x, kind_y, kind_z: ORC_AXIS_ODD or ORC_AXIS_EVEN (ignored for absent
 * axes).  z (three dimensions only) is periodic.
 * tau > 0 is used as given; tau <= 0 derives it from kn (Eq. kn) with the
 * wall distance H = ny (walls half way between nodes) in two and three
 * dimensions, or the domain length H = nx in one dimension; tau = +inf gives
 * omega = 0. */
orc_solver *orc_create3(int dims, int Lx, int Ly, int Lz, int kind_x, int kind_y, int kind_z, int64_t nx, int64_t ny,
                        int64_t nz, double tau, double kn, int bc_x, int bc_y, const double *wall_u,
                        const double *end_rho, double g)
{
    if (dims < 1 || dims > 3) return NULL;
    if (dims == 1) { Ly = 0; ny = 1; bc_y = ORC_BC_PERIODIC; kind_y = ORC_AXIS_ODD; }
    if (dims < 3) { Lz = 0; nz = 1; kind_z = ORC_AXIS_ODD; }
    if (Lx < 1 || (dims >= 2 && Ly < 1) || (dims == 3 && Lz < 1) || nx < 1 || ny < 1 || nz < 1) return NULL;
    if (Lx > 30 || Ly > 30 || Lz > 30) return NULL;
    if ((kind_x != ORC_AXIS_ODD && kind_x != ORC_AXIS_EVEN) || (kind_y != ORC_AXIS_ODD && kind_y != ORC_AXIS_EVEN) ||
        (kind_z != ORC_AXIS_ODD && kind_z != ORC_AXIS_EVEN))
        return NULL;
    if (bc_x != ORC_BC_PERIODIC && bc_x != ORC_BC_EQ_ENDS) return NULL;
    if (bc_y != ORC_BC_PERIODIC && bc_y != ORC_BC_WALL) return NULL;
    if (bc_x == ORC_BC_EQ_ENDS && bc_y == ORC_BC_WALL) return NULL;

    orc_solver *s = (orc_solver *)calloc(1, sizeof(orc_solver));
    s->dims = dims; s->Lx = Lx; s->Ly = Ly; s->Lz = Lz; s->nx = nx; s->ny = ny; s->nz = nz;
    s->kx = kind_x; s->ky = kind_y; s->kz = kind_z;
    s->bc_x = bc_x; s->bc_y = bc_y; s->g = g;
    s->wall_u[0] = wall_u ? wall_u[0] : 0.0; s->wall_u[1] = wall_u ? wall_u[1] : 0.0;
    s->end_rho[0] = end_rho ? end_rho[0] : 1.0; s->end_rho[1] = end_rho ? end_rho[1] : 1.0;
    s->Qx = axis_setup(kind_x, Lx, s->cx, &s->thx, &s->u2x);
    if (dims >= 2) {
        s->Qy = axis_setup(kind_y, Ly, s->cy, &s->thy, &s->u2y);
    } else {
        s->Qy = 1; s->cy[0] = 0; s->thy = 0.0; s->u2y = 0.0;
    }
    if (dims == 3) {
        s->Qz = axis_setup(kind_z, Lz, s->cz, &s->thz, &s->u2z);
    } else {
        s->Qz = 1; s->cz[0] = 0; s->thz = 0.0; s->u2z = 0.0;
    }
    s->Q = s->Qx * s->Qy * s->Qz;
    /* no population may cross both walls in one step */
    if (s->Q > 4096 || (bc_y == ORC_BC_WALL && ny < 2 * s->cy[s->Qy - 1])) {
        free(s);
        return NULL;
    }
    if (tau > 0.0) {
        s->tau = tau;
    } else {
        const double H = dims >= 2 ? (double)ny : (double)nx;
        const double th = dims >= 2 ? s->thy : s->thx;
        s->tau = orc_tau_from_kn(kn, H, th);
    }
    /* collision frequency Delta t / (tau + Delta t / 2), section 2 */
    s->omega = 1.0 / (s->tau + 0.5);

    s->Wx = (double *)calloc(s->Qx, sizeof(double));
    s->Wy = (double *)calloc(s->Qy, sizeof(double));
    s->Wz = (double *)calloc(s->Qz, sizeof(double));
    orc_axis_equilibrium(kind_x, Lx, 0.0, s->Wx);
    if (dims >= 2) orc_axis_equilibrium(kind_y, Ly, 0.0, s->Wy); else s->Wy[0] = 1.0;
    if (dims == 3) orc_axis_equilibrium(kind_z, Lz, 0.0, s->Wz); else s->Wz[0] = 1.0;
    s->Jplus_y = 0.0;
    for (int b = 0; b < s->Qy; ++b)
        if (s->cy[b] > 0) s->Jplus_y += s->cy[b] * s->Wy[b];

    s->Ebot = (double *)calloc(s->Q, sizeof(double));
    s->Etop = (double *)calloc(s->Q, sizeof(double));
    double *Fb = (double *)calloc(s->Qx, sizeof(double));
    double *Ft = (double *)calloc(s->Qx, sizeof(double));
    orc_axis_equilibrium(kind_x, Lx, s->wall_u[0], Fb);
    orc_axis_equilibrium(kind_x, Lx, s->wall_u[1], Ft);
    for (int c = 0; c < s->Qz; ++c)
        for (int b = 0; b < s->Qy; ++b)
            for (int a = 0; a < s->Qx; ++a) {
                const int q = (c * s->Qy + b) * s->Qx + a;
                s->Ebot[q] = Fb[a] * s->Wy[b] * s->Wz[c];
                s->Etop[q] = Ft[a] * s->Wy[b] * s->Wz[c];
            }
    free(Fb); free(Ft);

    const int64_t n = nodes(s);
    s->f = (double *)calloc((size_t)(s->Q * n), sizeof(double));
    s->fs = (double *)calloc((size_t)(s->Q * n), sizeof(double));
    s->fn = (double *)calloc((size_t)(s->Q * n), sizeof(double));
    s->ux_prev = (double *)calloc((size_t)n, sizeof(double));
    s->rw_bot = (double *)calloc((size_t)(nx * nz), sizeof(double));
    s->rw_top = (double *)calloc((size_t)(nx * nz), sizeof(double));
    s->t = 0;
    return s;
}

/* One or two dimensions (orc_create3 with no z axis). */
orc_solver *orc_create(int dims, int Lx, int Ly, int kind_x, int kind_y, int64_t nx, int64_t ny, double tau,
                       double kn, int bc_x, int bc_y, const double *wall_u, const double *end_rho, double g)
{
    if (dims != 1 && dims != 2) return NULL;
    return orc_create3(dims, Lx, Ly, 0, kind_x, kind_y, ORC_AXIS_ODD, nx, ny, 1, tau, kn, bc_x, bc_y, wall_u,
                       end_rho, g);
}

void orc_destroy(orc_solver *s)
{
    if (!s) return;
    free(s->Wx); free(s->Wy); free(s->Wz); free(s->Ebot); free(s->Etop);
    free(s->f); free(s->fs); free(s->fn); free(s->ux_prev);
    free(s->rw_bot); free(s->rw_top);
    free(s);
}

double orc_tau(const orc_solver *s) { return s->tau; }
double orc_omega(const orc_solver *s) { return s->omega; }
int64_t orc_time(const orc_solver *s) { return s->t; }
int orc_nvel(const orc_solver *s) { return s->Q; }

int orc_axis_velocities(const orc_solver *s, int *cx, int *cy)
{
    memcpy(cx, s->cx, sizeof(int) * s->Qx);
    memcpy(cy, s->cy, sizeof(int) * s->Qy);
    return s->Qx;
}

int orc_axis_velocities_z(const orc_solver *s, int *cz)
{
    memcpy(cz, s->cz, sizeof(int) * s->Qz);
    return s->Qz;
}

/* Rest weights of the two axes and the wall-normal half flux. */
void orc_tables(const orc_solver *s, double *Wx, double *Wy, double *jplus)
{
    memcpy(Wx, s->Wx, sizeof(double) * s->Qx);
    memcpy(Wy, s->Wy, sizeof(double) * s->Qy);
    *jplus = s->Jplus_y;
}

/* Tensor-product equilibrium (section 4):
 * f^eq_abc = rho F_a(u_x) F_b(u_y) F_c(u_z). */
static void equilibrium_node(const orc_solver *s, double rho, double ux, double uy, double uz, double *feq)
{
    double Fx[64], Fy[64], Fz[64];
    orc_axis_equilibrium(s->kx, s->Lx, ux, Fx);
    if (s->dims >= 2) orc_axis_equilibrium(s->ky, s->Ly, uy, Fy); else Fy[0] = 1.0;
    if (s->dims == 3) orc_axis_equilibrium(s->kz, s->Lz, uz, Fz); else Fz[0] = 1.0;
    for (int c = 0; c < s->Qz; ++c)
        for (int b = 0; b < s->Qy; ++b)
            for (int a = 0; a < s->Qx; ++a) feq[(c * s->Qy + b) * s->Qx + a] = rho * Fx[a] * Fy[b] * Fz[c];
}

/* f(0) = f^eq(rho, u) per node; uy and uz may be NULL (zero). */
void orc_init_fields3(orc_solver *s, const double *rho, const double *ux, const double *uy, const double *uz)
{
    const int64_t n = nodes(s);
    double feq[4096];
    for (int64_t k = 0; k < n; ++k) {
        equilibrium_node(s, rho ? rho[k] : 1.0, ux ? ux[k] : 0.0, uy ? uy[k] : 0.0, uz ? uz[k] : 0.0, feq);
        for (int q = 0; q < s->Q; ++q) s->f[q * n + k] = feq[q];
    }
    s->t = 0;
}

void orc_init_fields(orc_solver *s, const double *rho, const double *ux, const double *uy)
{
    orc_init_fields3(s, rho, ux, uy, NULL);
}

/* f(0) given directly, [q][z][y][x]. */
void orc_init_populations(orc_solver *s, const double *f0)
{
    memcpy(s->f, f0, sizeof(double) * (size_t)(s->Q * nodes(s)));
    s->t = 0;
}

void orc_get_populations(const orc_solver *s, double *out)
{
    memcpy(out, s->f, sizeof(double) * (size_t)(s->Q * nodes(s)));
}

/* Density and velocity of node k of a state (section 2 moment definitions). */
static void node_rho_u(const orc_solver *s, const double *f, int64_t k, double *rho, double *ux, double *uy,
                       double *uz)
{
    const int64_t n = nodes(s);
    double r = 0, jx = 0, jy = 0, jz = 0;
    for (int c = 0; c < s->Qz; ++c)
        for (int b = 0; b < s->Qy; ++b)
            for (int a = 0; a < s->Qx; ++a) {
                const double v = f[((c * s->Qy + b) * s->Qx + a) * n + k];
                r += v;
                jx += v * s->cx[a];
                jy += v * s->cy[b];
                jz += v * s->cz[c];
            }
    *rho = r; *ux = jx / r; *uy = jy / r; *uz = jz / r;
}

/* Collision of every node (Eq. maineq01 right-hand side plus the linear
 * force of section 5.4): f* = f + omega (f^eq - f) + F,
 * F_abc = W_a W_b W_c c_a g / theta_x, which adds momentum g and no mass. */
static void collide_all(const orc_solver *s, const double *f, double *fs, double *ux_out)
{
    const int64_t n = nodes(s);
    double feq[4096];
    for (int64_t k = 0; k < n; ++k) {
        double rho, ux, uy, uz;
        node_rho_u(s, f, k, &rho, &ux, &uy, &uz);
        if (ux_out) ux_out[k] = ux;
        equilibrium_node(s, rho, ux, uy, uz, feq);
        for (int c = 0; c < s->Qz; ++c)
            for (int b = 0; b < s->Qy; ++b)
                for (int a = 0; a < s->Qx; ++a) {
                    const int q = (c * s->Qy + b) * s->Qx + a;
                    const double force = s->Wx[a] * s->Wy[b] * s->Wz[c] * s->cx[a] * s->g / s->thx;
                    const double v = f[q * n + k];
                    fs[q * n + k] = v + s->omega * (feq[q] - v) + force;
                }
    }
}

/* Diffuse-reflection wall densities.  The paper cites the kinetic wall
 * condition without writing it out (sections 5.3, 5.4); the reading used
 * here: every post-collision population whose streaming would cross a wall
 * is absorbed and attributed to the column (x, z) it would have reached; the
 * wall re-emits that mass into the same column as the equilibrium at the
 * wall velocity, rho_w E_i, over the populations that point into the fluid,
 * so rho_w = absorbed / J+ with J+ = sum_{c>0} c W_c.  Arrays per column
 * are [z][x]. */
static void wall_densities(const orc_solver *s, const double *fs, double *rw_bot, double *rw_top,
                           double *mom_bot, double *mom_top)
{
    const int64_t n = nodes(s), nx = s->nx, ny = s->ny, nz = s->nz;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t x = 0; x < nx; ++x) {
            double ab = 0, at = 0, pb = 0, pt = 0;
            for (int c = 0; c < s->Qz; ++c) {
                const int64_t zs = imod(z - s->cz[c], nz);
                for (int b = 0; b < s->Qy; ++b) {
                    const int cb = s->cy[b];
                    for (int a = 0; a < s->Qx; ++a) {
                        const int ca = s->cx[a];
                        const int q = (c * s->Qy + b) * s->Qx + a;
                        const int64_t xs = imod(x - ca, nx);
                        if (cb < 0) {
                            for (int64_t y = 0; y < -cb; ++y) {
                                const double v = fs[q * n + (zs * ny + y) * nx + xs];
                                ab += v; pb += v * ca;
                            }
                        } else if (cb > 0) {
                            for (int64_t y = ny - cb; y < ny; ++y) {
                                const double v = fs[q * n + (zs * ny + y) * nx + xs];
                                at += v; pt += v * ca;
                            }
                        }
                    }
                }
            }
            rw_bot[z * nx + x] = ab / s->Jplus_y;
            rw_top[z * nx + x] = at / s->Jplus_y;
            if (mom_bot) mom_bot[z * nx + x] = pb;
            if (mom_top) mom_top[z * nx + x] = pt;
        }
}

/* Linear streaming (left-hand side of Eq. maineq01), written in pull form:
 * f_i(t+1, x) = f*_i(t, x - c_i), with the wall emission or the fixed
 * equilibrium ends where x - c_i lies outside the domain. */
static void stream_all(const orc_solver *s, const double *fs, double *fn)
{
    const int64_t n = nodes(s), nx = s->nx, ny = s->ny, nz = s->nz;
    for (int c = 0; c < s->Qz; ++c) {
        const int cc = s->cz[c];
        for (int b = 0; b < s->Qy; ++b) {
            const int cb = s->cy[b];
            for (int a = 0; a < s->Qx; ++a) {
                const int ca = s->cx[a];
                const int q = (c * s->Qy + b) * s->Qx + a;
                for (int64_t z = 0; z < nz; ++z) {
                    const int64_t zs = imod(z - cc, nz);
                    for (int64_t y = 0; y < ny; ++y)
                        for (int64_t x = 0; x < nx; ++x) {
                            int64_t ys = y - cb, xs = x - ca;
                            double v;
                            if (s->bc_y == ORC_BC_WALL && ys < 0) {
                                v = s->rw_bot[z * nx + x] * s->Ebot[q];
                            } else if (s->bc_y == ORC_BC_WALL && ys >= ny) {
                                v = s->rw_top[z * nx + x] * s->Etop[q];
                            } else {
                                ys = imod(ys, ny);
                                if (s->bc_x == ORC_BC_EQ_ENDS && xs < 0) {
                                    v = s->end_rho[0] * s->Wx[a] * s->Wy[b] * s->Wz[c];
                                } else if (s->bc_x == ORC_BC_EQ_ENDS && xs >= nx) {
                                    v = s->end_rho[1] * s->Wx[a] * s->Wy[b] * s->Wz[c];
                                } else {
                                    xs = imod(xs, nx);
                                    v = fs[q * n + (zs * ny + ys) * nx + xs];
                                }
                            }
                            fn[q * n + (z * ny + y) * nx + x] = v;
                        }
                }
            }
        }
    }
}

/* Advance nsteps time steps: collide, wall densities, stream. */
void orc_step(orc_solver *s, int64_t nsteps)
{
    for (int64_t it = 0; it < nsteps; ++it) {
        collide_all(s, s->f, s->fs, s->ux_prev);
        if (s->bc_y == ORC_BC_WALL) wall_densities(s, s->fs, s->rw_bot, s->rw_top, NULL, NULL);
        stream_all(s, s->fs, s->fn);
        double *tmp = s->f; s->f = s->fn; s->fn = tmp;
        s->t += 1;
    }
}

/* Moments of the pre-collision state f(t): rho, u, the temperature per
 * degree of freedom T = (sum f |c|^2 / rho - |u|^2) / D and the shear
 * moment Pxy = sum f c_x c_y - rho u_x u_y.  Any output may be NULL. */
void orc_moments3(const orc_solver *s, double *rho, double *ux, double *uy, double *uz, double *T, double *pxy)
{
    const int64_t n = nodes(s);
    for (int64_t k = 0; k < n; ++k) {
        double r = 0, jx = 0, jy = 0, jz = 0, exx = 0, eyy = 0, ezz = 0, exy = 0;
        for (int c = 0; c < s->Qz; ++c)
            for (int b = 0; b < s->Qy; ++b)
                for (int a = 0; a < s->Qx; ++a) {
                    const double v = s->f[((c * s->Qy + b) * s->Qx + a) * n + k];
                    const double ca = s->cx[a], cb = s->cy[b], cc = s->cz[c];
                    r += v; jx += v * ca; jy += v * cb; jz += v * cc;
                    exx += v * ca * ca; eyy += v * cb * cb; ezz += v * cc * cc; exy += v * ca * cb;
                }
        const double vx = jx / r, vy = jy / r, vz = jz / r;
        if (rho) rho[k] = r;
        if (ux) ux[k] = vx;
        if (uy) uy[k] = vy;
        if (uz) uz[k] = vz;
        if (T) T[k] = ((exx + eyy + ezz) / r - vx * vx - vy * vy - vz * vz) / s->dims;
        if (pxy) pxy[k] = exy - r * vx * vy;
    }
}

void orc_moments(const orc_solver *s, double *rho, double *ux, double *uy, double *T, double *pxy)
{
    orc_moments3(s, rho, ux, uy, NULL, T, pxy);
}

/* Kahan-compensated running sum. */
typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double v)
{
    const double y = v - k->c;
    const double t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

/* Global diagnostics at the current time t:
 *  out[0] mass        sum f(t)
 *  out[1] momentum x  sum f(t) c_x   (pre-collision)
 *  out[2] momentum y  sum f(t) c_y
 *  out[3] energy      sum f*(t) |c|^2 (post-collision; the model is
 *                     isothermal, so this is reported, not conserved)
 *  out[4] residual    ||u_x(t) - u_x(t-1)||_2 / ||u_x(t)||_2 (NaN at t = 0)
 *  out[5] absorbed mass at the bottom wall in the next streaming
 *  out[6] absorbed mass at the top wall
 *  out[7] x momentum given to the bottom wall in the next streaming
 *  out[8] x momentum given to the top wall
 *  out[9] number of nodes outside the positivity domain of section 3 on
 *         any axis (see axis_setup)
 *  out[10] momentum z  sum f(t) c_z
 *  out[11] number of nodes whose density, momentum or energy is not a
 *          finite number (failure detection; such a node is not counted in
 *          out[9], and it makes the sums above non-finite) */
void orc_stats(orc_solver *s, double *out)
{
    const int64_t n = nodes(s), ncol = s->nx * s->nz;
    ksum m = {0, 0}, px = {0, 0}, py = {0, 0}, pz = {0, 0}, e = {0, 0}, d2 = {0, 0}, u2 = {0, 0};
    double *ux = (double *)malloc(sizeof(double) * (size_t)n);
    collide_all(s, s->f, s->fs, ux);
    double npos = 0, nbad = 0;
    for (int64_t k = 0; k < n; ++k) {
        double r = 0, jx = 0, jy = 0, jz = 0, en = 0;
        for (int c = 0; c < s->Qz; ++c)
            for (int b = 0; b < s->Qy; ++b)
                for (int a = 0; a < s->Qx; ++a) {
                    const int q = (c * s->Qy + b) * s->Qx + a;
                    const double ca = s->cx[a], cb = s->cy[b], cc = s->cz[c];
                    const double v = s->f[q * n + k];
                    r += v; jx += v * ca; jy += v * cb; jz += v * cc;
                    en += s->fs[q * n + k] * (ca * ca + cb * cb + cc * cc);
                }
        kadd(&m, r); kadd(&px, jx); kadd(&py, jy); kadd(&pz, jz); kadd(&e, en);
        kadd(&u2, ux[k] * ux[k]);
        kadd(&d2, (ux[k] - s->ux_prev[k]) * (ux[k] - s->ux_prev[k]));
        const double vy = jy / r, vz = jz / r;
        if (!isfinite(r) || !isfinite(jx) || !isfinite(jy) || !isfinite(jz) || !isfinite(en))
            nbad += 1;
        else if (ux[k] * ux[k] > s->u2x || (s->dims >= 2 && vy * vy > s->u2y) || (s->dims == 3 && vz * vz > s->u2z))
            npos += 1;
    }
    out[0] = m.s; out[1] = px.s; out[2] = py.s; out[3] = e.s;
    out[4] = s->t > 0 ? sqrt(d2.s) / sqrt(u2.s) : NAN;
    out[5] = out[6] = out[7] = out[8] = 0.0;
    if (s->bc_y == ORC_BC_WALL) {
        double *pb = (double *)malloc(sizeof(double) * (size_t)ncol);
        double *pt = (double *)malloc(sizeof(double) * (size_t)ncol);
        double *rb = (double *)malloc(sizeof(double) * (size_t)ncol);
        double *rt = (double *)malloc(sizeof(double) * (size_t)ncol);
        wall_densities(s, s->fs, rb, rt, pb, pt);
        ksum ab = {0, 0}, at = {0, 0}, mb = {0, 0}, mt = {0, 0};
        for (int64_t x = 0; x < ncol; ++x) {
            const double Ab = rb[x] * s->Jplus_y, At = rt[x] * s->Jplus_y;
            kadd(&ab, Ab); kadd(&at, At);
            /* emitted x momentum per column is A U_w: the first moment of
             * the unit-density equilibrium at the wall velocity is U_w */
            kadd(&mb, pb[x] - Ab * s->wall_u[0]);
            kadd(&mt, pt[x] - At * s->wall_u[1]);
        }
        out[5] = ab.s; out[6] = at.s; out[7] = mb.s; out[8] = mt.s;
        free(pb); free(pt); free(rb); free(rt);
    }
    out[9] = npos;
    out[10] = pz.s;
    out[11] = nbad;
    free(ux);
}
