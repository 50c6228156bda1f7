// C-ABI of libglbm.so (declared in include/glbm.h): configuration checks,
// run-time tables, buffer bookkeeping and kernel dispatch.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/glbm.h"
#include "glbm_internal.h"

#include <map>

using namespace glbm;

namespace {

thread_local std::string g_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(GLBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

Variant g_variants[kAxisCodes][kAxisCodes][4][3][2];
std::once_flag g_once;

std::map<long long, Variant> g_variants3;

void register_all()
{
#define GLBM_CALL_REGISTER(E, C, L) register_##E##_##C##_##L();
    GLBM_OBJECTS(GLBM_CALL_REGISTER)
#undef GLBM_CALL_REGISTER
#define GLBM_CALL_REGISTER3(K) register3_##K();
    GLBM_OBJECTS3(GLBM_CALL_REGISTER3)
#undef GLBM_CALL_REGISTER3
}

// Host copy of the per-axis equilibrium at rho = 1 (N-fold convolution of the
// D1Q3 equilibrium at u/N, lattice units), in double, for the wall tables;
// the 2N+2 axis averages neighbouring pairs of the 2N+1 one at u/2.
void host_odd_equilibrium(int N, double u, double *F)
{
    double cur[kMaxQ1] = {1.0};
    int len = 1;
    const double v = u / N;
    const double pp = 1.0 / 6.0 + 0.5 * v + 0.5 * v * v;
    const double pm = 1.0 / 6.0 - 0.5 * v + 0.5 * v * v;
    const double p0 = 2.0 / 3.0 - v * v;
    for (int k = 0; k < N; ++k) {
        double nxt[kMaxQ1] = {};
        for (int i = 0; i < len; ++i) {
            nxt[i] += pm * cur[i];
            nxt[i + 1] += p0 * cur[i];
            nxt[i + 2] += pp * cur[i];
        }
        len += 2;
        for (int i = 0; i < len; ++i) cur[i] = nxt[i];
    }
    for (int i = 0; i < 2 * N + 1; ++i) F[i] = cur[i];
}

// Axis of code A (see Axis in glbm_device.h): velocities, reach, temperature.
struct HostAxis {
    int code, N, q, vmax;
    bool even;
    double theta;
};

HostAxis host_axis(int N, bool even)
{
    HostAxis a;
    a.N = N;
    a.even = even;
    a.code = N == 0 ? 0 : even ? kEven + N : N;
    a.q = N == 0 ? 1 : even ? 2 * N + 2 : 2 * N + 1;
    a.vmax = even ? 2 * N + 1 : N;
    a.theta = even ? (4.0 * N + 3.0) / 3.0 : N / 3.0;
    return a;
}

void host_axis_equilibrium(const HostAxis &ax, double u, double *F)
{
    if (!ax.even) {
        host_odd_equilibrium(ax.N, u, F);
        return;
    }
    double G[kMaxQ1];
    host_odd_equilibrium(ax.N, 0.5 * u, G);
    for (int a = 0; a <= 2 * ax.N + 1; ++a)
        F[a] = 0.5 * ((a >= 1 ? G[a - 1] : 0.0) + (a <= 2 * ax.N ? G[a] : 0.0));
}

struct Geometry {
    HostAxis x, y, z;
    int q, eb;
    int bcx;  // kernel variant's x boundary and row layout (BcX)
    int64_t nx, ny, nz, nxp;  // rows are numbered z ny + y
    uint64_t plane_bytes, buf_bytes;
};

int check_config(const glbm_config *c, Geometry *g)
{
    if (!c) return fail(GLBM_ERR_INVALID, "config is NULL");
    if (c->dims < 1 || c->dims > 3) return fail(GLBM_ERR_INVALID, "dims must be 1, 2 or 3 (got %d)", c->dims);
    const int lx = c->level_x, ly = c->dims >= 2 ? c->level_y : 0, lz = c->dims == 3 ? c->level_z : 0;
    // levels up to kMaxLevel pass here; the kernels built for each lattice
    // (7 per axis, 13 for the even axis of the mixed channel lattices) are
    // checked at glbm_create
    if (lx < 1 || lx > kMaxLevel) return fail(GLBM_ERR_INVALID, "level_x must be in 1..%d", kMaxLevel);
    if (c->dims >= 2 && (ly < 1 || ly > kMaxLevel)) return fail(GLBM_ERR_INVALID, "level_y must be in 1..%d", kMaxLevel);
    if (c->dims == 3 && (lz < 1 || lz > kMaxLevel)) return fail(GLBM_ERR_INVALID, "level_z must be in 1..%d", kMaxLevel);
    const int kx = c->kind_x, ky = c->dims >= 2 ? c->kind_y : GLBM_AXIS_ODD, kz = c->dims == 3 ? c->kind_z : GLBM_AXIS_ODD;
    if ((kx != GLBM_AXIS_ODD && kx != GLBM_AXIS_EVEN) || (ky != GLBM_AXIS_ODD && ky != GLBM_AXIS_EVEN) ||
        (kz != GLBM_AXIS_ODD && kz != GLBM_AXIS_EVEN))
        return fail(GLBM_ERR_INVALID, "axis kinds must be GLBM_AXIS_ODD or GLBM_AXIS_EVEN");
    const HostAxis ax = host_axis(lx, kx == GLBM_AXIS_EVEN), ay = host_axis(ly, ky == GLBM_AXIS_EVEN);
    const HostAxis az = host_axis(lz, kz == GLBM_AXIS_EVEN);
    if (c->storage < GLBM_STORE_F32 || c->storage > GLBM_STORE_BF16_SHIFTED_SR)
        return fail(GLBM_ERR_INVALID, "unknown storage %d", c->storage);
    const int64_t nx = c->nx, ny = c->dims >= 2 ? c->ny : 1, nz = c->dims == 3 ? c->nz : 1;
    if (nx < 1 || ny < 1 || nz < 1) return fail(GLBM_ERR_INVALID, "nx, ny and nz must be positive");
    if (c->dims == 3 && c->bc_x != GLBM_BC_PERIODIC)
        return fail(GLBM_ERR_INVALID, "three-dimensional lattices are periodic in x");
    if (c->dims == 3 && nz < az.vmax)
        return fail(GLBM_ERR_INVALID, "nz (%lld) must be at least the fastest z velocity %d", (long long)nz, az.vmax);
    if (c->bc_x != GLBM_BC_PERIODIC && c->bc_x != GLBM_BC_EQ_ENDS)
        return fail(GLBM_ERR_INVALID, "bc_x must be periodic or equilibrium ends");
    const int bcy = c->dims >= 2 ? c->bc_y : GLBM_BC_PERIODIC;
    if (bcy != GLBM_BC_PERIODIC && bcy != GLBM_BC_WALL)
        return fail(GLBM_ERR_INVALID, "bc_y must be periodic or wall");
    if (c->bc_x == GLBM_BC_EQ_ENDS && bcy == GLBM_BC_WALL)
        return fail(GLBM_ERR_INVALID, "walls and equilibrium ends cannot be combined");
    // no population may cross both walls (or wrap more than once across y) in
    // one step
    if (bcy == GLBM_BC_WALL && ny < 2 * ay.vmax)
        return fail(GLBM_ERR_INVALID, "ny (%lld) must be at least 2*%d (twice the fastest y velocity) with walls",
                    (long long)ny, ay.vmax);
    if (c->dims >= 2 && bcy == GLBM_BC_PERIODIC && ny < ay.vmax)
        return fail(GLBM_ERR_INVALID, "periodic ny (%lld) must be at least the fastest y velocity %d", (long long)ny,
                    ay.vmax);
    if (c->bc_x == GLBM_BC_EQ_ENDS && nx < ax.vmax)
        return fail(GLBM_ERR_INVALID, "nx must be at least the fastest x velocity with equilibrium ends");
    // round to nearest loses every per-step increment below half a BF16 unit
    // of the deviation: a driven flow (force or walls) stalls far from the
    // solution, so the storage is offered for undriven lattices only
    if (c->storage == GLBM_STORE_BF16_SHIFTED && (c->g != 0.0 || bcy == GLBM_BC_WALL))
        return fail(GLBM_ERR_UNSUPPORTED,
                    "round-to-nearest BF16 storage stalls driven flows (force or walls): use the stochastic "
                    "rounding storage");
    g->x = ax;
    g->y = ay;
    g->z = az;
    g->q = ax.q * ay.q * az.q;
    g->eb = (c->storage == GLBM_STORE_BF16_SHIFTED || c->storage == GLBM_STORE_BF16_SHIFTED_SR) ? 2 : 4;
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    // two and three dimensions (periodic x): compact rows of nx columns (node
    // x at column x, the x wrap taken per lane in the pull); one dimension:
    // padded rows with ghosts (node x at column kGhost + x)
    const bool compact = c->dims >= 2 && c->bc_x == GLBM_BC_PERIODIC;
    g->bcx = compact ? BCX_WRAP : c->bc_x == GLBM_BC_EQ_ENDS ? BCX_EQ : BCX_PERIODIC;
    g->nxp = compact ? nx : (kGhost + nx + ax.vmax + 63) / 64 * 64;
    g->plane_bytes = ((uint64_t)(nz * ny * g->nxp) * g->eb + 255) & ~(uint64_t)255;
    g->buf_bytes = (g->plane_bytes * g->q + 255) & ~(uint64_t)255;
    if (nx * ny * nz > (int64_t)0x7fffffff / 4) return fail(GLBM_ERR_INVALID, "too many nodes");
    if (g->buf_bytes >= ((uint64_t)1 << 32))
        return fail(GLBM_ERR_INVALID, "population buffer of %llu bytes exceeds 4 GiB", (unsigned long long)g->buf_bytes);
    return GLBM_OK;
}

__global__ void bump_counter(int64_t *c, int64_t k) { *c += k; }

__global__ void reduce_partials(const double *partials, int nblocks, double *out)
{
    __shared__ double red[kBlock];
    for (int k = 0; k < kNumStats; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += kBlock) s += partials[(size_t)b * kNumStats + k];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = red[0];
        __syncthreads();
    }
}

}  // namespace

namespace glbm {
Variant *variant_slot(int ax, int ay, int storage, int bcx, int bcy)
{
    return &g_variants[ax][ay][storage][bcx][bcy];
}

Variant *variant3_slot(int ax, int ay, int az, int storage, int bcx, int bcy)
{
    const long long key = ((((long long)ax * kAxisCodes + ay) * kAxisCodes + az) * 4 + storage) * 6 + bcx * 2 + bcy;
    return &g_variants3[key];
}
}  // namespace glbm

struct glbm_solver {
    glbm_config cfg;
    Geometry geo;
    double tau, omega;
    void *buf[2];
    int cur;  // index of the buffer holding f*(t); the other holds f*(t-1) or f(0)
    int64_t t;
    bool ready;
    hipStream_t stream;
    const Variant *var;
    KArgs base;
    int grid;
    double *d_partials, *d_out, *h_out;
    float *d_wrate;  // walls: per-column wall factors of a step
    int device;
    bool in_batch;
};

extern "C" {

const char *glbm_last_error(void) { return g_error.c_str(); }

size_t glbm_population_bytes(const glbm_config *cfg)
{
    Geometry g;
    if (check_config(cfg, &g) != GLBM_OK) return 0;
    return (size_t)g.buf_bytes;
}

// Rows of FP64 partial sums of one statistics launch (the blocks stride over
// the nodes), and the bytes of a solver's statistics buffers.
static int stat_blocks(int64_t nodes)
{
    const int64_t g = (nodes + kBlock - 1) / kBlock;
    return (int)std::min<int64_t>(g, kStatBlocks);
}

static size_t stats_bytes(int64_t nodes)
{
    return sizeof(double) * kNumStats * ((size_t)stat_blocks(nodes) + 1);
}

// The kernel variant of a valid configuration (its step is null if not built).
static const Variant *variant_of(const glbm_config *cfg, const Geometry &g)
{
    std::call_once(g_once, register_all);
    const int bcy = cfg->dims >= 2 ? cfg->bc_y : GLBM_BC_PERIODIC;
    return cfg->dims == 3 ? variant3_slot(g.x.code, g.y.code, g.z.code, cfg->storage, g.bcx, bcy)
                          : variant_slot(g.x.code, g.y.code, cfg->storage, g.bcx, bcy);
}

// Bytes of the wall factors of a variant whose step reads them (the bottom
// and top factor of every column (x, z), written by the wall pre-pass of a
// step: three-dimensional lattices and the largest symmetric ones with
// walls), 0 otherwise.
static size_t wrate_bytes(const Variant *v, const Geometry &g)
{
    return v->wall_rates ? 2 * sizeof(float) * (size_t)(g.nx * g.nz) : 0;
}

size_t glbm_required_bytes(const glbm_config *cfg)
{
    Geometry g;
    if (check_config(cfg, &g) != GLBM_OK) return 0;
    return 2 * (size_t)g.buf_bytes + stats_bytes(g.nx * g.ny * g.nz) + wrate_bytes(variant_of(cfg, g), g);
}

int glbm_create(const glbm_config *cfg, void *pop_a, void *pop_b, void *stream, glbm_t **out)
{
    if (!out) return fail(GLBM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    Geometry g;
    int rc = check_config(cfg, &g);
    if (rc != GLBM_OK) return rc;
    if (!pop_a || !pop_b || pop_a == pop_b) return fail(GLBM_ERR_INVALID, "two distinct population buffers are required");
    if (((uintptr_t)pop_a & 255) || ((uintptr_t)pop_b & 255)) return fail(GLBM_ERR_INVALID, "buffers must be 256-byte aligned");

    double tau = cfg->tau;
    if (!(tau > 0.0)) {
        const double H = cfg->dims >= 2 ? (double)g.ny : (double)g.nx;
        const double theta = cfg->dims >= 2 ? g.y.theta : g.x.theta;
        if (!(cfg->kn > 0.0)) return fail(GLBM_ERR_INVALID, "either tau > 0 or kn > 0 is required");
        tau = cfg->kn * H / sqrt(2.0 * theta);  // Eq. kn with nu = theta tau
    }
    const double omega = 1.0 / (tau + 0.5);
    if (!(omega > 0.0 && omega < 2.0)) return fail(GLBM_ERR_INVALID, "collision frequency %g outside (0, 2)", omega);

    const int bcy = cfg->dims >= 2 ? cfg->bc_y : GLBM_BC_PERIODIC;
    const Variant *v = variant_of(cfg, g);
    if (!v->step)
        return fail(GLBM_ERR_UNSUPPORTED, "no kernels built for axes (%s%d, %s%d, %s%d) with these boundaries",
                    g.x.even ? "even " : "", g.x.N, g.y.even ? "even " : "", g.y.N, g.z.even ? "even " : "", g.z.N);

    glbm_solver *h = new (std::nothrow) glbm_solver();
    if (!h) return fail(GLBM_ERR_INVALID, "out of host memory");
    h->cfg = *cfg;
    h->geo = g;
    h->tau = tau;
    h->omega = omega;
    h->buf[0] = pop_a;
    h->buf[1] = pop_b;
    h->cur = 0;
    h->t = 0;
    h->ready = false;
    h->in_batch = false;
    h->stream = (hipStream_t)stream;
    h->var = v;
    (void)hipGetDevice(&h->device);

    const int64_t nodes = g.nx * g.ny * g.nz;
    h->grid = (int)((nodes + kBlock - 1) / kBlock);
    KArgs &a = h->base;
    memset(&a, 0, sizeof a);
    a.buf_bytes = (uint32_t)g.buf_bytes;
    a.plane_bytes = (uint32_t)g.plane_bytes;
    a.nx = (int32_t)g.nx;
    a.ny = (int32_t)g.ny;
    a.nz = (int32_t)g.nz;
    a.nxp = (int32_t)g.nxp;
    a.nodes = (int32_t)nodes;
    a.remap = 1;
    a.omega = (float)omega;
    a.gth = (float)(cfg->g / g.x.theta);  // force shape W_a c_a g / theta_x
    a.g = (float)cfg->g;
    // wall emission: unit-density equilibrium at the wall speed (x) times the
    // rest weights (y), in FP32; the kernels divide the absorbed mass by the
    // mass these FP32 tables emit, so that each column keeps its mass
    double F[kMaxQ1];
    for (int side = 0; side < 2; ++side) {
        const double U = bcy == GLBM_BC_WALL ? cfg->wall_u[side] : 0.0;
        host_axis_equilibrium(g.x, U, F);
        double sum = 0.0;
        for (int i = 0; i < g.x.q; ++i) {
            a.fw[side][i] = (float)F[i];
            sum += (double)a.fw[side][i];
        }
        a.fwsum[side] = sum;
        a.uw[side] = (float)U;
    }

    if (const size_t wb = wrate_bytes(v, g)) {
        hipError_t e = hipMalloc((void **)&h->d_wrate, wb);
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "allocating the wall factors");
        }
        a.wrate = h->d_wrate;
    }
    // the FP64 statistics buffers are allocated by the first glbm_stats call,
    // so that a solver that never asks for them costs no device allocation
    *out = h;
    return GLBM_OK;
}

static int do_init(glbm_t *h, const float *rho, const float *ux, const float *uy, const float *uz, const float *f0)
{
    if (!h) return fail(GLBM_ERR_INVALID, "handle is NULL");
    KArgs a = h->base;
    hipError_t e;
    if (h->cfg.bc_x == GLBM_BC_EQ_ENDS) {
        a.dst = h->buf[0];
        a.dst2 = h->buf[1];
        const int n = h->geo.q * (int)h->geo.ny * 2 * h->geo.x.vmax;
        e = h->var->ends(a, (n + kBlock - 1) / kBlock, (float)h->cfg.end_rho[0], (float)h->cfg.end_rho[1], h->stream);
        if (e != hipSuccess) return hip_fail(e, "launching the end-state fill");
    }
    a.dst = h->buf[0];   // f*(0)
    a.dst2 = h->buf[1];  // f(0)
    a.i_rho = rho;
    a.i_ux = ux;
    a.i_uy = uy;
    a.i_uz = uz;
    a.i_f = f0;
    a.seed = step_seed(0);
    e = h->var->init(a, h->grid, h->stream);
    if (e != hipSuccess) return hip_fail(e, "launching the init kernel");
    h->cur = 0;
    h->t = 0;
    h->ready = true;
    return GLBM_OK;
}

int glbm_init_fields(glbm_t *h, const float *rho, const float *ux, const float *uy)
{
    return do_init(h, rho, ux, uy, nullptr, nullptr);
}

int glbm_init_fields3(glbm_t *h, const float *rho, const float *ux, const float *uy, const float *uz)
{
    return do_init(h, rho, ux, uy, uz, nullptr);
}

int glbm_init_populations(glbm_t *h, const float *f0)
{
    if (!f0) return fail(GLBM_ERR_INVALID, "f0 is NULL");
    return do_init(h, nullptr, nullptr, nullptr, nullptr, f0);
}

int glbm_step(glbm_t *h, int64_t nsteps)
{
    if (!h) return fail(GLBM_ERR_INVALID, "handle is NULL");
    if (!h->ready) return fail(GLBM_ERR_STATE, "step before init");
    if (h->in_batch) return fail(GLBM_ERR_STATE, "the solver belongs to a batch: step the batch");
    if (nsteps < 0) return fail(GLBM_ERR_INVALID, "nsteps must be >= 0");
    KArgs a = h->base;
    for (int64_t s = 0; s < nsteps; ++s) {
        a.src = h->buf[h->cur];
        a.dst = h->buf[1 - h->cur];
        a.seed = step_seed(h->t + 1);
        hipError_t e = h->var->step(a, h->grid, h->stream);
        if (e != hipSuccess) return hip_fail(e, "launching the step kernel");
        h->cur = 1 - h->cur;
        h->t += 1;
    }
    return GLBM_OK;
}

static int observe(glbm_t *h, float *rho, float *ux, float *uy, float *uz, float *T, float *pxy, float *f)
{
    if (!h) return fail(GLBM_ERR_INVALID, "handle is NULL");
    if (!h->ready) return fail(GLBM_ERR_STATE, "moments before init");
    KArgs a = h->base;
    // f(t) is the pull of f*(t-1) (t >= 1) or the stored f(0) itself (t = 0);
    // both live in the buffer that the next step will overwrite.
    a.src = h->buf[1 - h->cur];
    a.local = h->t == 0;
    a.o_rho = rho;
    a.o_ux = ux;
    a.o_uy = uy;
    a.o_uz = uz;
    a.o_T = T;
    a.o_pxy = pxy;
    a.o_f = f;
    hipError_t e = h->var->observe(a, h->grid, h->stream);
    if (e != hipSuccess) return hip_fail(e, "launching the observe kernel");
    return GLBM_OK;
}

int glbm_moments(glbm_t *h, float *rho, float *ux, float *uy, float *T, float *pxy)
{
    return observe(h, rho, ux, uy, nullptr, T, pxy, nullptr);
}

int glbm_moments3(glbm_t *h, float *rho, float *ux, float *uy, float *uz, float *T, float *pxy)
{
    return observe(h, rho, ux, uy, uz, T, pxy, nullptr);
}

int glbm_get_populations(glbm_t *h, float *out)
{
    if (!out) return fail(GLBM_ERR_INVALID, "out is NULL");
    return observe(h, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, out);
}

// Statistics of h into *out through the FP64 buffers partials (stat_blocks
// rows) and dout (kNumStats values) on the device and hout on the host;
// synchronizes the stream.  Returns the failure status of the state.
static int stats_through(glbm_t *h, double *partials, double *dout, double *hout, glbm_stats_t *out)
{
    KArgs a = h->base;
    a.src = h->buf[h->cur];
    a.prev = h->t > 0 ? h->buf[1 - h->cur] : nullptr;
    a.partials = partials;
    const int blocks = stat_blocks((int64_t)a.nodes);
    hipError_t e = h->var->stats(a, blocks, h->stream);
    if (e != hipSuccess) return hip_fail(e, "launching the stats kernel");
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kBlock), 0, h->stream, partials, blocks, dout);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "launching the reduction");
    e = hipMemcpyAsync(hout, dout, sizeof(double) * kNumStats, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "reading the statistics");
    const double *s = hout;
    out->time = h->t;
    out->mass = s[0];
    out->momentum_x = s[1];
    out->momentum_y = s[2];
    out->energy_post = s[3];
    out->residual = h->t > 0 ? sqrt(s[5]) / sqrt(s[4]) : NAN;
    out->wall_mass[0] = s[6];
    out->wall_momentum[0] = s[7];
    out->wall_mass[1] = s[8];
    out->wall_momentum[1] = s[9];
    out->nonpositive_nodes = s[10];
    out->momentum_z = s[11];
    out->nonfinite_nodes = s[12];
    if (s[12] > 0)
        return fail(GLBM_ERR_NONFINITE, "%.0f nodes have a non-finite density, momentum or energy at t = %lld", s[12],
                    (long long)h->t);
    if (s[10] > 0)
        return fail(GLBM_ERR_POSITIVITY, "%.0f nodes are outside the positivity domain of the equilibrium at t = %lld",
                    s[10], (long long)h->t);
    return GLBM_OK;
}

int glbm_stats(glbm_t *h, glbm_stats_t *out)
{
    if (!h || !out) return fail(GLBM_ERR_INVALID, "NULL argument");
    if (!h->ready) return fail(GLBM_ERR_STATE, "stats before init");
    hipError_t e = hipSuccess;
    if (!h->d_partials) {
        const size_t rows = (size_t)stat_blocks((int64_t)h->base.nodes);
        e = hipMalloc((void **)&h->d_partials, sizeof(double) * kNumStats * rows);
        if (e == hipSuccess) e = hipMalloc((void **)&h->d_out, sizeof(double) * kNumStats);
        if (e == hipSuccess) e = hipHostMalloc((void **)&h->h_out, sizeof(double) * kNumStats, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipFree(h->d_partials);
            (void)hipFree(h->d_out);
            h->d_partials = nullptr;
            h->d_out = nullptr;
            h->h_out = nullptr;
            return hip_fail(e, "allocating statistics buffers");
        }
    }
    return stats_through(h, h->d_partials, h->d_out, h->h_out, out);
}

int glbm_info(const glbm_t *h, double *tau, double *omega, int32_t *nvel, int64_t *time)
{
    if (!h) return fail(GLBM_ERR_INVALID, "handle is NULL");
    if (tau) *tau = h->tau;
    if (omega) *omega = h->omega;
    if (nvel) *nvel = h->geo.q;
    if (time) *time = h->t;
    return GLBM_OK;
}

int glbm_destroy(glbm_t *h)
{
    if (!h) return GLBM_OK;
    if (h->in_batch) return fail(GLBM_ERR_STATE, "the solver belongs to a batch: destroy the batch first");
    // kernels may still use these buffers
    if (h->d_partials || h->d_wrate) (void)hipStreamSynchronize(h->stream);
    if (h->d_partials) {
        (void)hipFree(h->d_partials);
        (void)hipFree(h->d_out);
        (void)hipHostFree(h->h_out);
    }
    if (h->d_wrate) (void)hipFree(h->d_wrate);
    delete h;
    return GLBM_OK;
}


}  // extern "C"

// ------------------------------------------ statistics without allocation
// glbm_stats_static: glbm_stats for callers that cannot allocate device
// memory.  The partial sums and totals go through `scratch`, a file-scope
// device array that every GPU the library runs on holds once (it stays
// allocated until the process ends).  Host code never passes the array's name
// to a kernel or copy: it uses the device address hipGetSymbolAddress gives
// for the current device, fetched once per device and kept.
constexpr int kScratchRows = kStatBlocks + 1;  // partial-sum rows, then the totals
static __device__ __align__(256) double scratch[kScratchRows * kNumStats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (made current for the lookup).
int scratch_on(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(GLBM_ERR_INVALID, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void *ptr = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "locating the statistics scratch");
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return GLBM_OK;
}
}  // namespace

extern "C" int glbm_stats_static(glbm_t *h, glbm_stats_t *out)
{
    if (!h || !out) return fail(GLBM_ERR_INVALID, "NULL argument");
    if (!h->ready) return fail(GLBM_ERR_STATE, "stats before init");
    const int blocks = stat_blocks((int64_t)h->base.nodes);
    if (blocks + 1 > kScratchRows)
        return fail(GLBM_ERR_INVALID, "statistics need %d partial rows, the scratch holds %d", blocks, kScratchRows - 1);
    double *ptr = nullptr;
    const int rc = scratch_on(h->device, &ptr);
    if (rc != GLBM_OK) return rc;
    double hout[kNumStats];
    // every block writes its whole row and the reduction writes every total,
    // so nothing in the scratch needs clearing between calls
    return stats_through(h, ptr, ptr + (size_t)kStatBlocks * kNumStats, hout, out);
}
// ------------------------------------------ end of statistics without allocation

// ------------------------------------------------------------------ batches
//
// All device tables of a batch live in one allocation, uploaded from a
// pinned host copy with one asynchronous copy on the batch's stream:
//   [step counter int64][phase int32 x n][t0 int64 x n][args KArgs x 2n]
//   [tiles of each (variant, row set)][resident member lists of each variant]
// Re-planning (glbm_batch_update) rewrites them in place; the allocation
// grows (by doubling) only when a plan does not fit.

struct glbm_batch {
    struct RowSet {
        const Variant *var;
        int rows;        // StepRows
        size_t tiles;    // byte offset of the set's tiles in the table block
        int ntiles;
    };
    glbm_batch_options opt;
    struct ResidentSet {
        const Variant *var;
        size_t list;     // byte offset of the member indices in the table block
        int count;
    };
    std::vector<glbm_solver *> members;
    std::vector<RowSet> sets;
    std::vector<ResidentSet> resident;
    hipStream_t user;  // caller's stream (may be NULL)
    hipStream_t exec;  // stream the batch launches on
    bool own_stream;
    hipEvent_t ev_in, ev_out, ev_staged;
    char *d_mem, *h_mem;  // device tables and their pinned host copy
    size_t cap;           // bytes of each
    size_t o_phase, o_t0, o_args;
    hipGraph_t graph;
    hipGraphExec_t graph_exec;
    bool planned;  // the tables match `members`
    // side streams for the variants (opt.streams - 1 of them), the fork event
    // recorded on exec and one join event per side stream
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_done;
    hipEvent_t ev_fork;
};

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static void release_graph(glbm_batch *b)
{
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
}

static void batch_free(glbm_batch *b)
{
    release_graph(b);
    (void)hipFree(b->d_mem);
    (void)hipHostFree(b->h_mem);
    if (b->ev_staged) (void)hipEventDestroy(b->ev_staged);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->own_stream) (void)hipStreamDestroy(b->exec);
    for (auto ev : b->side_done) (void)hipEventDestroy(ev);
    for (auto st : b->side) (void)hipStreamDestroy(st);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (auto *m : b->members) m->in_batch = false;
    delete b;
}

template <class T>
static T *at(char *base, size_t off)
{
    return reinterpret_cast<T *>(base + off);
}

// One chunk of k steps: for each kernel variant, its resident launch and
// launches l = 0..k-1 of its row sets, then the device step counter advances
// by k.  Variants hold disjoint members, so they need no ordering between
// them: with side streams, variant v runs on stream v mod S (the batch's
// stream first), forked from and joined back into the batch's stream.
static hipError_t batch_chunk(glbm_batch *b, int k)
{
    int64_t *bstep = at<int64_t>(b->d_mem, 0);
    const int32_t *phase = at<int32_t>(b->d_mem, b->o_phase);
    const int64_t *t0 = at<int64_t>(b->d_mem, b->o_t0);
    const KArgs *args = at<KArgs>(b->d_mem, b->o_args);
    std::vector<const Variant *> vars;
    for (auto &r : b->resident)
        if (std::find(vars.begin(), vars.end(), r.var) == vars.end()) vars.push_back(r.var);
    for (auto &r : b->sets)
        if (std::find(vars.begin(), vars.end(), r.var) == vars.end()) vars.push_back(r.var);
    const size_t S = std::min(b->side.size() + 1, vars.size());
    hipError_t e = hipSuccess;
    if (S > 1) {
        e = hipEventRecord(b->ev_fork, b->exec);
        for (size_t i = 0; e == hipSuccess && i + 1 < S; ++i) e = hipStreamWaitEvent(b->side[i], b->ev_fork, 0);
        if (e != hipSuccess) return e;
    }
    for (size_t v = 0; v < vars.size(); ++v) {
        const size_t si = v % S;
        hipStream_t st = si == 0 ? b->exec : b->side[si - 1];
        for (auto &r : b->resident)
            if (r.var == vars[v]) {
                e = r.var->resident(at<int32_t>(b->d_mem, r.list), r.count, args, phase, t0, bstep, k, st);
                if (e != hipSuccess) return e;
            }
        for (int l = 0; l < k; ++l)
            for (auto &r : b->sets)
                if (r.var == vars[v]) {
                    e = r.var->batch(r.rows, at<BatchTile>(b->d_mem, r.tiles), r.ntiles, b->opt.tile_nodes, args,
                                     phase, t0, bstep, l, st);
                    if (e != hipSuccess) return e;
                }
    }
    for (size_t i = 0; e == hipSuccess && i + 1 < S; ++i) {
        e = hipEventRecord(b->side_done[i], b->side[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->exec, b->side_done[i], 0);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bump_counter, dim3(1), dim3(1), 0, b->exec, bstep, (int64_t)k);
    return hipGetLastError();
}

// Check a prospective member list (members of `self` may stay; an update may
// empty the batch).
static int check_members(glbm_t *const *members, int32_t n, const glbm_batch *self)
{
    if (self ? (n < 0 || (n > 0 && !members)) : (!members || n < 1))
        return fail(GLBM_ERR_INVALID, "a batch needs at least one member");
    for (int i = 0; i < n; ++i) {
        glbm_solver *m = members[i];
        if (!m) return fail(GLBM_ERR_INVALID, "member %d is NULL", i);
        if (!m->ready) return fail(GLBM_ERR_STATE, "member %d is not initialised", i);
        if (!m->var->batch) return fail(GLBM_ERR_UNSUPPORTED, "member %d: its lattice has no batched step", i);
        const bool mine = self && std::find(self->members.begin(), self->members.end(), m) != self->members.end();
        if (m->in_batch && !mine) return fail(GLBM_ERR_STATE, "member %d already belongs to a batch", i);
        for (int j = 0; j < i; ++j)
            if (members[j] == m) return fail(GLBM_ERR_INVALID, "member %d appears twice", i);
    }
    return GLBM_OK;
}

// Lay out the tables for `members` in the pinned host copy (growing both
// copies if needed), upload them on the batch's stream and re-capture the
// graph.  On failure the batch is left without a valid plan.
static int plan(glbm_batch *b, glbm_t *const *members, int32_t n)
{
    b->planned = false;
    struct Part {
        int member, count;
        double work;
    };
    const int tile = b->opt.tile_nodes;
    auto is_resident = [&](const glbm_solver *m) {
        return b->opt.resident_nodes > 0 && m->var->resident &&
               m->geo.nx * m->geo.ny * m->geo.nz <= (int64_t)b->opt.resident_nodes;
    };
    std::vector<const Variant *> vars;
    for (int i = 0; i < n; ++i)
        if (std::find(vars.begin(), vars.end(), members[i]->var) == vars.end()) vars.push_back(members[i]->var);
    // resident member lists per variant
    std::vector<glbm_batch::ResidentSet> rsets;
    std::vector<std::vector<int32_t>> rlists;
    for (const Variant *v : vars) {
        std::vector<int32_t> ids;
        for (int i = 0; i < n; ++i)
            if (members[i]->var == v && is_resident(members[i])) ids.push_back(i);
        if (ids.empty()) continue;
        rsets.push_back({v, 0, (int)ids.size()});
        rlists.push_back(std::move(ids));
    }
    // tile lists per (variant, row set)
    std::vector<glbm_batch::RowSet> sets;
    std::vector<std::vector<BatchTile>> lists;
    for (const Variant *v : vars) {
        const int rowsets[2][2] = {{ROWS_INTERIOR, ROWS_WALLS}, {ROWS_ALL, -1}};
        for (int rsi = 0; rsi < 2; ++rsi) {
            const int rows = rowsets[v->split_rows ? 0 : 1][rsi];
            if (rows < 0) break;
            std::vector<Part> parts;
            for (int i = 0; i < n; ++i) {
                const glbm_solver *m = members[i];
                if (m->var != v || is_resident(m)) continue;
                const int64_t nx = m->geo.nx, ny = m->geo.ny, ly = m->geo.y.vmax;  // rows with wall emission
                const int64_t cnt = rows == ROWS_ALL ? nx * ny * m->geo.nz
                                    : rows == ROWS_INTERIOR ? (ny - 2 * ly) * nx : 2 * ly * nx;
                if (cnt > 0) parts.push_back({i, (int)cnt, (double)cnt * m->geo.q});
            }
            if (b->opt.order == GLBM_ORDER_LARGEST_FIRST)
                std::stable_sort(parts.begin(), parts.end(), [](const Part &x, const Part &y) { return x.work > y.work; });
            std::vector<BatchTile> tiles;
            if (b->opt.order == GLBM_ORDER_INTERLEAVE) {
                for (int first = 0;; first += tile) {
                    bool any = false;
                    for (const Part &pt : parts)
                        if (first < pt.count) {
                            tiles.push_back({pt.member, first, std::min(tile, pt.count - first), 0});
                            any = true;
                        }
                    if (!any) break;
                }
            } else {
                for (const Part &pt : parts)
                    for (int first = 0; first < pt.count; first += tile)
                        tiles.push_back({pt.member, first, std::min(tile, pt.count - first), 0});
            }
            if (tiles.empty()) continue;
            sets.push_back({v, rows, 0, (int)tiles.size()});
            lists.push_back(std::move(tiles));
        }
    }
    // layout
    size_t off = 256;
    b->o_phase = off;
    off = align_up(off + sizeof(int32_t) * n, 256);
    b->o_t0 = off;
    off = align_up(off + sizeof(int64_t) * n, 256);
    b->o_args = off;
    off = align_up(off + sizeof(KArgs) * 2 * (size_t)n, 256);
    for (size_t k = 0; k < sets.size(); ++k) {
        sets[k].tiles = off;
        off = align_up(off + sizeof(BatchTile) * lists[k].size(), 256);
    }
    for (size_t k = 0; k < rsets.size(); ++k) {
        rsets[k].list = off;
        off = align_up(off + sizeof(int32_t) * rlists[k].size(), 256);
    }
    const size_t need = off;
    b->sets.clear();
    b->resident.clear();
    release_graph(b);

    // the previous upload must have left the pinned copy before it is rewritten
    hipError_t e = hipEventSynchronize(b->ev_staged);
    if (e == hipSuccess && need > b->cap) {
        size_t cap = std::max<size_t>(need, 2 * b->cap);
        e = hipStreamSynchronize(b->exec);
        if (e == hipSuccess) {
            (void)hipFree(b->d_mem);
            (void)hipHostFree(b->h_mem);
            b->d_mem = nullptr;
            b->h_mem = nullptr;
            b->cap = 0;
            e = hipMalloc((void **)&b->d_mem, cap);
            if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_mem, cap, hipHostMallocDefault);
            if (e == hipSuccess) b->cap = cap;
        }
    }
    if (e != hipSuccess) return hip_fail(e, "allocating the batch tables");

    char *h = b->h_mem;
    *at<int64_t>(h, 0) = 0;
    for (int i = 0; i < n; ++i) {
        const glbm_solver *m = members[i];
        at<int32_t>(h, b->o_phase)[i] = m->cur;
        at<int64_t>(h, b->o_t0)[i] = m->t;
        for (int c = 0; c < 2; ++c) {
            KArgs a = m->base;
            a.src = m->buf[c];
            a.dst = m->buf[1 - c];
            a.remap = 0;
            at<KArgs>(h, b->o_args)[2 * i + c] = a;
        }
    }
    for (size_t k = 0; k < sets.size(); ++k)
        memcpy(h + sets[k].tiles, lists[k].data(), sizeof(BatchTile) * lists[k].size());
    for (size_t k = 0; k < rsets.size(); ++k)
        memcpy(h + rsets[k].list, rlists[k].data(), sizeof(int32_t) * rlists[k].size());
    e = hipMemcpyAsync(b->d_mem, h, need, hipMemcpyHostToDevice, b->exec);
    if (e == hipSuccess) e = hipEventRecord(b->ev_staged, b->exec);
    if (e != hipSuccess) return hip_fail(e, "uploading the batch tables");
    b->sets = std::move(sets);
    b->resident = std::move(rsets);

    if (b->opt.graph_steps > 0 && (!b->sets.empty() || !b->resident.empty())) {
        e = hipStreamBeginCapture(b->exec, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t ec = batch_chunk(b, b->opt.graph_steps);
            e = hipStreamEndCapture(b->exec, &b->graph);
            if (ec != hipSuccess) e = ec;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            b->sets.clear();
            b->resident.clear();
            release_graph(b);
            return hip_fail(e, "capturing the batch graph");
        }
    }
    b->planned = true;
    return GLBM_OK;
}

static void set_members(glbm_batch *b, glbm_t *const *members, int32_t n)
{
    for (auto *m : b->members) m->in_batch = false;
    b->members.assign(members, members + n);
    for (auto *m : b->members) m->in_batch = true;
}

extern "C" {

int glbm_batch_create(glbm_t *const *members, int32_t n, const glbm_batch_options *opt, void *stream,
                      glbm_batch_t **out)
{
    if (!out) return fail(GLBM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    glbm_batch_options o = {256, GLBM_ORDER_MEMBER, 0, 0, 1};
    if (opt) o = *opt;
    if (o.tile_nodes == 0) o.tile_nodes = 256;
    if (o.streams == 0) o.streams = 1;
    if (o.streams < 1 || o.streams > 8) return fail(GLBM_ERR_INVALID, "streams must be 1..8");
    if (o.tile_nodes != 64 && o.tile_nodes != 128 && o.tile_nodes != 256)
        return fail(GLBM_ERR_INVALID, "tile_nodes must be 64, 128 or 256");
    if (o.order < GLBM_ORDER_MEMBER || o.order > GLBM_ORDER_LARGEST_FIRST)
        return fail(GLBM_ERR_INVALID, "unknown tile order");
    if (o.graph_steps < 0) return fail(GLBM_ERR_INVALID, "graph_steps must be >= 0");
    if (o.resident_nodes < 0) return fail(GLBM_ERR_INVALID, "resident_nodes must be >= 0");
    int rc = check_members(members, n, nullptr);
    if (rc != GLBM_OK) return rc;

    glbm_batch *b = new (std::nothrow) glbm_batch();
    if (!b) return fail(GLBM_ERR_INVALID, "out of host memory");
    b->opt = o;
    b->user = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (b->user) {
        b->exec = b->user;
    } else {
        e = hipStreamCreateWithFlags(&b->exec, hipStreamNonBlocking);
        b->own_stream = e == hipSuccess;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_staged, hipEventDisableTiming);
    if (e == hipSuccess && o.streams > 1) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    for (int i = 1; e == hipSuccess && i < o.streams; ++i) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) b->side.push_back(st);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) b->side_done.push_back(ev);
    }
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "creating the batch streams");
    }
    rc = plan(b, members, n);
    if (rc != GLBM_OK) {
        batch_free(b);
        return rc;
    }
    set_members(b, members, n);
    *out = b;
    return GLBM_OK;
}

int glbm_batch_update(glbm_batch_t *b, glbm_t *const *members, int32_t n)
{
    if (!b) return fail(GLBM_ERR_INVALID, "batch is NULL");
    int rc = check_members(members, n, b);
    if (rc != GLBM_OK) return rc;
    rc = plan(b, members, n);
    if (rc != GLBM_OK) {
        // keep the old members owned (their state is intact) but unplanned:
        // stepping fails until a successful update
        return rc;
    }
    set_members(b, members, n);
    return GLBM_OK;
}

int glbm_batch_step(glbm_batch_t *b, int64_t nsteps)
{
    if (!b) return fail(GLBM_ERR_INVALID, "batch is NULL");
    if (nsteps < 0) return fail(GLBM_ERR_INVALID, "nsteps must be >= 0");
    if (!b->planned) return fail(GLBM_ERR_STATE, "the batch has no valid plan (a previous update failed)");
    if (nsteps == 0 || b->members.empty()) return GLBM_OK;
    hipError_t e = hipSuccess;
    if (b->own_stream) {
        // order after the caller's earlier work on the default stream
        e = hipEventRecord(b->ev_in, b->user);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->exec, b->ev_in, 0);
    }
    int64_t left = nsteps;
    while (e == hipSuccess && b->graph_exec && left >= b->opt.graph_steps) {
        e = hipGraphLaunch(b->graph_exec, b->exec);
        left -= b->opt.graph_steps;
    }
    while (e == hipSuccess && left > 0) {
        const int k = (int)std::min<int64_t>(left, 1 << 20);
        e = batch_chunk(b, k);
        left -= k;
    }
    if (e == hipSuccess && b->own_stream) {
        e = hipEventRecord(b->ev_out, b->exec);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->user, b->ev_out, 0);
    }
    if (e != hipSuccess) return hip_fail(e, "stepping the batch");
    for (auto *m : b->members) {
        m->t += nsteps;
        if (nsteps & 1) m->cur = 1 - m->cur;
    }
    return GLBM_OK;
}

int glbm_batch_destroy(glbm_batch_t *b)
{
    if (!b) return GLBM_OK;
    (void)hipStreamSynchronize(b->exec);
    batch_free(b);
    return GLBM_OK;
}

}  // extern "C"
