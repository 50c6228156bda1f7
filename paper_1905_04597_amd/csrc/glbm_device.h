// Device code of the Gaussian lattice Boltzmann hierarchy for gfx950.
//
// One lane owns one lattice node and keeps all Q populations of that node in
// registers for the whole step:
//   pull (Eq. maineq01 streaming, read side) -> moments (section 2) ->
//   per-axis equilibrium = N-fold convolution of the D1Q3 equilibrium at
//   u/N (Eqs. maineq02-maineq06 in lattice units) -> tensor product
//   (section 4) -> BGK relaxation with collision frequency 1/(tau + 1/2)
//   plus the linear force of section 5.4 -> store.
//
// Memory layout of a population buffer: velocity planes [q][row][column].
//
// Two- and three-dimensional lattices (periodic x) use compact rows of
// exactly nx columns (rows y, or z * ny + y): each plane is one contiguous
// run of nodes, so that consecutive workgroups stream consecutive bytes of
// every plane whatever nx is.  The pull computes the source column
// (x - c_x) mod nx once per x velocity, a per-lane register; the y and z
// shifts are whole rows.  (Padded rows with ghost columns measured slower
// here: the ghosts and the row padding break the planes into short runs.)
//
// One-dimensional lattices use one padded row of nxp columns (a multiple of
// 64); node x lives at column x + G, G = 64.  The columns within reach of the
// fastest x velocity on each side of the interior are ghosts.  With periodic
// x every store of an edge node is replicated into the matching ghost
// columns, so a pull never wraps: the source of velocity c_x sits at a
// constant byte shift from the node, which the buffer loads take as an
// immediate offset.  With fixed equilibrium ends the ghosts hold the end
// state and are never written.
//
// Tables that depend only on the level (rest weights, half flux, force
// shape) are compile-time constants folded into the instructions; tables
// that depend on run-time parameters (wall emission at the wall speed) are
// kernel arguments, uniform across the wave and held in scalar registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace glbm {

// Largest level of an axis: 7 for every lattice, 13 for the G-D1Q(2N+2) axis
// across the walls of the mixed channel lattices (G-D1Q28 x D1Q3 at N = 13,
// the lattice of the Knudsen minimum in section 5.4).
constexpr int kMaxLevel = 13;
constexpr int kMaxQ1 = 2 * kMaxLevel + 2;  // velocities of the largest axis
constexpr int kBlock = 256;
constexpr int kNumStats = 13;
constexpr int kGhost = 64;  // padded column of node x = 0 (>= the largest level)

enum StorageKind { ST_F32 = 0, ST_F32S = 1, ST_BF16S = 2, ST_BF16SR = 3 };
// x boundary and row layout: periodic x with ghost columns (padded rows, one
// dimension), periodic x in compact rows (rows of exactly nx columns, the
// pull wraps; two and three dimensions), fixed equilibrium ends (padded rows
// whose ghosts hold the ends).
enum BcX { BCX_PERIODIC = 0, BCX_WRAP = 1, BCX_EQ = 2 };
enum BcY { BCY_PERIODIC = 0, BCY_WALL = 1 };

// ------------------------------------------------------------------ axes
// An axis is named by a code A.  A = N (1..7): the G-D1Q(2N+1) axis of level
// N, velocities -N..N, temperature N/3 (section 2 with unit lattice step).
// A = kEven + N: the G-D1Q(2N+2) axis of level N with the zero velocity
// removed (section 2, Eqs. maineq01_noball-maineq04_noball): its velocities
// (n + 1/2) c are laid on a grid of half the lattice step c, so they are the
// odd integers -(2N+1)..2N+1, and its temperature is (4N+3) c^2 / 12 =
// (4N+3)/3 (Eq. temp_2N2 with c = 2).  A = 0: the absent y axis of a
// one-dimensional lattice (the single velocity 0).
constexpr int kEven = 16;
constexpr int kAxisCodes = 2 * kEven;

template <int A>
struct Axis {
    static constexpr bool even = A > kEven;
    static constexpr int N = even ? A - kEven : A;
    static constexpr int Q = A == 0 ? 1 : even ? 2 * N + 2 : 2 * N + 1;
    static constexpr int vmax = even ? 2 * N + 1 : N;  // largest |c|: rows or columns one step reaches
    static constexpr int cmin = even ? 1 : 0;          // smallest |c|
    static constexpr int c(int a) { return even ? 2 * a - (2 * N + 1) : a - N; }
    static constexpr double theta = even ? (4.0 * N + 3.0) / 3.0 : N / 3.0;
    // positivity (section 3): the underlying 2N+1 walk keeps P0 >= 0 while
    // u^2 <= 2 N theta0, theta0 = N s^2 / 3 for its lattice step s (1, or 2
    // on the half grid of an even axis)
    static constexpr double u2max = 2.0 * N * N / 3.0 * (even ? 4.0 : 1.0);
};

// ---------------------------------------------------------------- tables
// Rest weights of an axis: the equilibrium at rho = 1, u = 0.  Level N:
// the coefficients of (1/6 z^-1 + 2/3 + 1/6 z)^N (N-fold sum of D1Q3 at
// rest, section 2 and Appendix A); the 2N+2 axis takes half of each
// neighbouring pair of those.  Computed in double at compile time and made
// exactly symmetric.
template <int A>
struct RestWeights {
    double w[Axis<A>::Q];
    constexpr RestWeights() : w{}
    {
        constexpr int N = Axis<A>::N;
        double cur[2 * kMaxLevel + 1] = {};
        cur[0] = 1.0;
        int len = 1;
        for (int k = 0; k < N; ++k) {
            double nxt[2 * kMaxLevel + 1] = {};
            for (int i = 0; i < len; ++i) {
                nxt[i] += cur[i] / 6.0;
                nxt[i + 1] += cur[i] * (2.0 / 3.0);
                nxt[i + 2] += cur[i] / 6.0;
            }
            len += 2;
            for (int i = 0; i < len; ++i) cur[i] = nxt[i];
        }
        for (int i = 0; i < N; ++i) cur[2 * N - i] = cur[i];
        if constexpr (Axis<A>::even) {
            for (int a = 0; a <= 2 * N + 1; ++a)
                w[a] = 0.5 * ((a >= 1 ? cur[a - 1] : 0.0) + (a <= 2 * N ? cur[a] : 0.0));
        } else {
            for (int a = 0; a <= 2 * N; ++a) w[a] = cur[a];
        }
    }
};

template <int A>
inline constexpr RestWeights<A> kRest{};

// Half flux J+ = sum_{c>0} c W_c of the FP32-rounded rest weights (exact sum).
template <int A>
constexpr double half_flux_f32()
{
    double s = 0.0;
    for (int a = 0; a < Axis<A>::Q; ++a)
        if (Axis<A>::c(a) > 0) s += Axis<A>::c(a) * (double)(float)kRest<A>.w[a];
    return s;
}

// The shift of the shifted storages is snapped to the 2^-24 grid (exact in
// FP32 below 1) with the centre entry absorbing the remainder, so that it sums
// to exactly one: rho = 1 + sum of deviations is then exact and the FP32
// collision carries no systematic mass error, only unbiased rounding.  (The
// shift is only an offset; tables that stand for physical weights keep full
// relative FP32 precision instead.)
constexpr double kGrid = 16777216.0;  // 2^24

constexpr long long snap(double w) { return (long long)(w * kGrid + 0.5); }

// Shift of the shifted storages: S_ab ~ W_a W_b on the grid, symmetric; the
// rounding remainder goes to the slowest populations (|c_x|, |c_y| smallest:
// 1, 2 or 4 of them) in equal parts, so the sum is exactly 1 when the
// remainder divides evenly (always with a zero velocity on both axes) and
// otherwise 1 - r 2^-24 (r < 4), which FP32 holds exactly: rho = sum +
// sum of deviations.  Plus the moments of S that the kernels add back.
template <int LX, int LY>
struct ShiftTable {
    static constexpr int QX = Axis<LX>::Q, QY = Axis<LY>::Q;
    float s[QY][QX];
    float sum;             // sum of S
    float sxx, syy;        // sum S c_x^2, sum S c_y^2
    float absorbed;        // sum of S over the populations one wall absorbs per column
    constexpr ShiftTable() : s{}, sum(0.0f), sxx(0.0f), syy(0.0f), absorbed(0.0f)
    {
        long long q[QY][QX] = {};
        long long tot = 0;
        for (int b = 0; b < QY; ++b)
            for (int a = 0; a < QX; ++a) tot += (q[b][a] = snap(kRest<LX>.w[a] * kRest<LY>.w[b]));
        const long long m = (Axis<LX>::even ? 2 : 1) * (Axis<LY>::even ? 2 : 1);
        const long long rem = (long long)kGrid - tot;
        const long long share = rem >= 0 ? rem / m : -((-rem + m - 1) / m);  // floor(rem / m)
        long long all = 0, xx = 0, yy = 0, ab = 0;
        for (int b = 0; b < QY; ++b)
            for (int a = 0; a < QX; ++a) {
                const long long ca = Axis<LX>::c(a), cb = Axis<LY>::c(b);
                if ((ca < 0 ? -ca : ca) == Axis<LX>::cmin && (cb < 0 ? -cb : cb) == Axis<LY>::cmin) q[b][a] += share;
                all += q[b][a];
                xx += q[b][a] * ca * ca;
                yy += q[b][a] * cb * cb;
                if (cb < 0) ab += q[b][a] * (-cb);
                s[b][a] = (float)(q[b][a] / kGrid);
            }
        sum = (float)(all / kGrid);
        sxx = (float)(xx / kGrid);
        syy = (float)(yy / kGrid);
        absorbed = (float)(ab / kGrid);
    }
};

template <int LX, int LY>
inline constexpr ShiftTable<LX, LY> kShift{};

// ------------------------------------------------------- unroll helper
template <int I, int E, class F>
__device__ __forceinline__ void unroll_from(F &&f)
{
    if constexpr (I < E) {
        f(std::integral_constant<int, I>{});
        unroll_from<I + 1, E>(f);
    }
}
template <int E, class F>
__device__ __forceinline__ void unroll(F &&f)
{
    unroll_from<0, E>(f);
}

// ------------------------------------------------------------- storage
template <int ST>
struct Elem;
template <>
struct Elem<ST_F32> {
    static constexpr int bytes = 4;
    static constexpr bool shifted = false;
};
template <>
struct Elem<ST_F32S> {
    static constexpr int bytes = 4;
    static constexpr bool shifted = true;
};
template <>
struct Elem<ST_BF16S> {
    static constexpr int bytes = 2;
    static constexpr bool shifted = true;
};
template <>
struct Elem<ST_BF16SR> {
    static constexpr int bytes = 2;
    static constexpr bool shifted = true;
};

using rsrc_t = __amdgpu_buffer_rsrc_t;

// Cache policy of the population stores: non-temporal (each value is written
// once per step and read by other waves only in the next launch).  The loads
// keep the default policy: neighbouring tiles re-read the halo lines from L2.
constexpr int kStoreNT = 2;
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    // raw buffer (stride 0), gfx9-family dword 3
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

template <int ST>
__device__ __forceinline__ float ld(rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (Elem<ST>::bytes == 2) {
        auto raw = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
        return __builtin_bit_cast(float, ((uint32_t)__builtin_bit_cast(unsigned short, raw)) << 16);
    } else {
        // the builtin returns the raw 32 bits as an integer
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    }
}

// Store one value; `rnd` is 32 random bits for the stochastic rounding mode.
template <int ST>
__device__ __forceinline__ void st(rsrc_t r, uint32_t voff, uint32_t soff, float v, uint32_t rnd = 0)
{
    if constexpr (ST == ST_BF16S) {
        const __bf16 h = (__bf16)v;  // round to nearest even (v_cvt_pk_bf16_f32)
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, h), r, voff, soff, kStoreNT);
    } else if constexpr (ST == ST_BF16SR) {
        // stochastic rounding in hardware (v_cvt_sr_bf16_f32): unbiased, so
        // increments far below one bf16 ulp still accumulate on average
        bf16x2_t h = {};
        h = __builtin_amdgcn_cvt_sr_bf16_f32(h, v, rnd, false);
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)__builtin_bit_cast(uint32_t, h), r, voff, soff, kStoreNT);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, kStoreNT);
    }
}

// 32-bit integer mixer (xor-shift-multiply, "lowbias32" constants).
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// Random bits of population q at a node whose hash is h: a rotation of h
// (distinct 32-bit windows for q mod 32), decorrelated across groups of 32.
template <int q>
__device__ __forceinline__ uint32_t rnd_of(uint32_t h)
{
    constexpr uint32_t rot = q & 31;
    uint32_t r = rot ? __builtin_amdgcn_alignbit(h, h, rot) : h;
    if constexpr ((q >> 5) != 0) r ^= (uint32_t)(q >> 5) * 0x9e3779b9U;
    return r;
}

// The value a 16-bit storage keeps of v (same rounding as st()).
template <int ST>
__device__ __forceinline__ float quantize(float v, uint32_t rnd)
{
    if constexpr (ST == ST_BF16S) {
        const __bf16 h = (__bf16)v;
        return __builtin_bit_cast(float, (uint32_t)__builtin_bit_cast(unsigned short, h) << 16);
    } else if constexpr (ST == ST_BF16SR) {
        bf16x2_t h = {};
        h = __builtin_amdgcn_cvt_sr_bf16_f32(h, v, rnd, false);
        return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, h) << 16);
    } else {
        return v;
    }
}

// ------------------------------------------------------------ kernel args
struct KArgs {
    const void *src;      // pull source: post-collision f*(t-1) (or f(0) in local mode)
    void *dst;            // destination of f*(t)
    uint32_t buf_bytes;   // bytes of one population buffer
    uint32_t plane_bytes; // bytes of one velocity plane (ny * nxp elements)
    int32_t nx, ny, nxp;  // nodes per axis, row length (padded: a multiple of 64 with ghosts; compact: nx)
    int32_t nz;           // nodes along z (three dimensions; 1 otherwise)
    int32_t nodes;        // nx * ny
    int32_t remap;        // XCD-aware block order
    int32_t local;        // observe kernel: read f(t) at the node, no streaming
    uint32_t seed;        // per-step seed of the stochastic rounding
    float omega;          // 1 / (tau + 1/2)
    float gth;            // g / theta_x
    float fw[2][kMaxQ1];  // F_a(U_wall) at unit density (FP32), bottom / top wall
    double fwsum[2];      // sum_a fw_a of the FP32 table (exact, in double)
    // observe outputs (canonical [y][x] / [q][y][x], may be null)
    float *o_rho, *o_ux, *o_uy, *o_T, *o_pxy, *o_f;
    float *o_uz;          // three dimensions
    // stats
    const void *prev;     // f*(t-1) for the residual (null at t = 0)
    float g;
    float uw[2];          // wall velocities
    double *partials;     // [gridDim][kNumStats]
    // init
    const float *i_rho, *i_ux, *i_uy, *i_f;
    const float *i_uz;    // three dimensions
    void *dst2;           // init: buffer receiving f(0)
    // walls: the wall factors of this step per column (x, z), bottom [nz][nx]
    // then top (nz = 1 in two dimensions), from the wall pre-pass
    float *wrate;
};

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous run of tiles so that the halo lines two neighbouring tiles share
// meet in the same L2.
__device__ __forceinline__ int tile_of(int b, int G, int remap)
{
    if (!remap) return b;
    const int G8 = G & ~7;
    if (b >= G8) return b;
    return (b & 7) * (G8 >> 3) + (b >> 3);
}
__device__ __forceinline__ int tile_index(const KArgs &p) { return tile_of(blockIdx.x, gridDim.x, p.remap); }

// ------------------------------------------------- per-axis equilibrium
// F_n(u), n = -N..N: N-fold convolution of the D1Q3 equilibrium at v = u/N,
// i.e. of the step probabilities of Eq. maineq04 with c = 1, theta = N/3:
// p+- = 1/6 +- v/2 + v^2/2 and p0 = 1 - p+ - p-.
template <int N, class T = float>
__device__ __forceinline__ void odd_equilibrium(T u, T (&F)[2 * N + 1])
{
    if constexpr (N == 0) {
        F[0] = T(1);
    } else {
        const T v = u / (T)N;
        const T hv = T(0.5) * v;
        const T pp = hv * (v + T(1)) + T(1) / T(6);
        const T pm = hv * (v - T(1)) + T(1) / T(6);
        const T p0 = (T(1) - pp) - pm;
        F[0] = pm;
        F[1] = p0;
        F[2] = pp;
        // multiply by (pm z^-1 + p0 + pp z) once per further level, in place
        // from the top entry down (entry j reads entries j, j-1, j-2 of the
        // previous level)
        unroll<N - 1>([&](auto K) {
            constexpr int k = K + 2;  // level being built; the previous has 2k-1 entries
            unroll<2 * k + 1>([&](auto J) {
                constexpr int j = 2 * k - (int)J;
                T s = T(0);
                if constexpr (j <= 2 * k - 2) s = pm * F[j];
                if constexpr (j >= 1 && j - 1 <= 2 * k - 2) s = p0 * F[j - 1] + s;
                if constexpr (j >= 2) s = pp * F[j - 2] + s;
                F[j] = s;
            });
        });
    }
}

// Equilibrium of axis A at rho = 1.  The 2N+2 axis (half grid, c = 2): the
// 2N+1 equilibrium of lattice step 2 at u, which is the unit-step one at
// u / 2, each velocity (n + 1/2) c taking half of its two neighbours n c and
// (n + 1) c (Eqs. maineq01_noball-maineq04_noball).
template <int A, class T = float>
__device__ __forceinline__ void axis_equilibrium(T u, T (&F)[Axis<A>::Q])
{
    constexpr int N = Axis<A>::N;
    if constexpr (!Axis<A>::even) {
        odd_equilibrium<N, T>(u, F);
    } else {
        T G[2 * N + 1];
        odd_equilibrium<N, T>(T(0.5) * u, G);
        F[0] = T(0.5) * G[0];
        unroll<2 * N>([&](auto J) {
            constexpr int j = J + 1;
            F[j] = T(0.5) * (G[j - 1] + G[j]);
        });
        F[2 * N + 1] = T(0.5) * G[2 * N];
    }
}

// ------------------------------------------------------------ the pull
// Working value of a population: f itself (plain storage) or its deviation
// f - S_ab from the rest state (shifted storage).
template <int LX, int LY, int ST>
struct Lat {
    static constexpr int QX = Axis<LX>::Q, QY = Axis<LY>::Q, Q = QX * QY;
    static constexpr int EB = Elem<ST>::bytes;
    static constexpr bool shifted = Elem<ST>::shifted;
};

// Byte offsets of the x sources of node x within a row (see the layouts
// above).  Padded rows: the source of velocity index a is column G + x - c_x,
// a constant shift that the load takes as an immediate.  Compact rows: column
// (x - c_x) mod nx, one register per velocity.
template <int LX, int EB, int BCX>
struct XAddr {
    static constexpr int QX = Axis<LX>::Q, V = Axis<LX>::vmax;
    static constexpr bool compact = BCX == BCX_WRAP;
    uint32_t col[compact ? QX : 1];
    uint32_t self;
    __device__ __forceinline__ XAddr(int x, int nx)
    {
        if constexpr (compact) {
            unroll<QX>([&](auto A) {
                constexpr int ca = Axis<LX>::c(A);
                int c = x - ca;
                if constexpr (ca > 0)
                    while (c < 0) c += nx;
                if constexpr (ca < 0)
                    while (c >= nx) c -= nx;
                col[A] = (uint32_t)c * (uint32_t)EB;
            });
            self = (uint32_t)x * (uint32_t)EB;
        } else {
            col[0] = (uint32_t)(x + kGhost - V) * (uint32_t)EB;
            self = (uint32_t)(x + kGhost) * (uint32_t)EB;
        }
    }
    // source of velocity index a in the row that starts at byte rowb
    template <int a>
    __device__ __forceinline__ uint32_t src(uint32_t rowb) const
    {
        if constexpr (compact)
            return rowb + col[a];
        else
            return rowb + col[0] + (uint32_t)((V - Axis<LX>::c(a)) * EB);
    }
    __device__ __forceinline__ uint32_t own(uint32_t rowb) const { return rowb + self; }
    // The same address split into a per-lane part and a uniform part: padded
    // rows keep one register per row and move the constant column shift to
    // the scalar offset (which the loads add anyway), so that no address
    // register per velocity is needed where the compiler does not fold the
    // shift into the immediate offset.
    template <int a>
    __device__ __forceinline__ uint32_t src_lane(uint32_t rowb) const
    {
        if constexpr (compact)
            return rowb + col[a];
        else
            return rowb + col[0];
    }
    template <int a>
    static constexpr uint32_t src_uniform()
    {
        return compact ? 0u : (uint32_t)((V - Axis<LX>::c(a)) * EB);
    }
};

template <int EB>
__device__ __forceinline__ uint32_t row_bytes(const KArgs &p, int row)
{
    return (uint32_t)(row * p.nxp) * (uint32_t)EB;
}

// Mass absorbed by a diffuse wall in column x: the post-collision
// populations that leave through the wall in this streaming and would land in
// column x (sources at x - c_x in the rows within reach of the wall).  The
// wall re-emits it into column x as rho_w(x) = A(x) / J+ times the
// unit-density equilibrium at the wall speed over the populations pointing
// into the fluid, which conserves the mass of every column.  `mom` receives
// the x momentum of the absorbed populations when requested.
template <int LX, int LY, int ST, int BCX, bool BOTTOM>
__device__ __forceinline__ float wall_absorbed(const KArgs &p, rsrc_t rs, const XAddr<LX, Elem<ST>::bytes, BCX> &xa,
                                               float *mom)
{
    using L = Lat<LX, LY, ST>;
    float s = 0.0f, m = 0.0f;
    unroll<L::QY>([&](auto B) {
        constexpr int b = B, cb = Axis<LY>::c(b);
        if constexpr ((BOTTOM && cb < 0) || (!BOTTOM && cb > 0)) {
            constexpr int depth = cb < 0 ? -cb : cb;
            unroll<depth>([&](auto R) {
                const int row = BOTTOM ? (int)R : p.ny - 1 - (int)R;
                const uint32_t rowb = row_bytes<L::EB>(p, row);
                unroll<L::QX>([&](auto A) {
                    constexpr int a = A, ca = Axis<LX>::c(a);
                    const float v = ld<ST>(rs, xa.template src<a>(rowb), (uint32_t)(b * L::QX + a) * p.plane_bytes);
                    s += v;
                    if (mom) m = __builtin_fmaf((float)ca, v, m);
                });
            });
        }
    });
    if (mom) *mom = m;  // the shift is even in c_x: it carries no x momentum
    if constexpr (L::shifted) s += kShift<LX, LY>.absorbed;
    return s;
}

// Wall re-emission factor of column x: rho_w / (J+ sum_a fw_a), J+ the mass
// the FP32 emission tables give out per unit wall density.
template <int LX, int LY, int ST, int BCX, bool BOTTOM>
__device__ __forceinline__ float wall_factor(const KArgs &p, rsrc_t rs, const XAddr<LX, Elem<ST>::bytes, BCX> &xa)
{
    constexpr double jp = half_flux_f32<LY>();
    return wall_absorbed<LX, LY, ST, BCX, BOTTOM>(p, rs, xa, nullptr) / (float)(jp * p.fwsum[BOTTOM ? 0 : 1]);
}

// Whether the single-lattice step with walls reads the wall factors from a
// pre-pass (wall_rate_kernel: once per column) rather than have every lane of
// the 2R wall rows sum its column (QX R (R + 1) / 2 loads): where the wall
// rows are a one-wave launch of their own (split lattices, above 144
// velocities) and that sum is at least twice the node's own loads, i.e. the
// symmetric G-D1Q(2N+2) products at N = 6 and 7 (G-D2Q256: 1920 loads per
// wall-row lane against 256; 1829 -> 1707 us in FP32, 1300 -> 1081 us in
// BF16).  Elsewhere the sums mostly hit L2 next to a wave-rich launch, and
// the extra launch per step measured 2-8% slower (D1Q3 x G-D1Q(2N+2),
// N = 2..12).
template <int LX, int LY, int ST>
constexpr bool wall_prepass()
{
    return Lat<LX, LY, ST>::Q > 144 && Axis<LY>::vmax * (Axis<LY>::vmax + 1) >= 4 * Axis<LY>::Q;
}

// Pre-collision populations of node (x, y) at the new time: pulled from the
// source buffer, or emitted by a wall where the source row is outside.
// INTERIOR: the node is at least the fastest y velocity away from both walls,
// so nothing is emitted into it and the pull has no branches.  PRE: the wall
// factors of column x come from the pre-pass of this step (the same
// arithmetic).
template <int LX, int LY, int ST, int BCX, int BCY, bool INTERIOR = false, bool PRE = false>
__device__ __forceinline__ void pull(const KArgs &p, rsrc_t rs, const XAddr<LX, Elem<ST>::bytes, BCX> &xa, int x, int y,
                                     float (&v)[Axis<LY>::Q][Axis<LX>::Q])
{
    using L = Lat<LX, LY, ST>;
    float rw[2] = {0.0f, 0.0f};
    if constexpr (BCY == BCY_WALL && !INTERIOR) {
        constexpr int reach = Axis<LY>::vmax;  // rows that take wall emission
        if constexpr (PRE) {
            if (y < reach) rw[0] = p.wrate[x];
            if (y >= p.ny - reach) rw[1] = p.wrate[p.nx + x];
        } else {
            if (y < reach) rw[0] = wall_factor<LX, LY, ST, BCX, true>(p, rs, xa);
            if (y >= p.ny - reach) rw[1] = wall_factor<LX, LY, ST, BCX, false>(p, rs, xa);
        }
    }
    unroll<L::QY>([&](auto B) {
        constexpr int b = B, cb = Axis<LY>::c(b);
        int ys = y - cb;
        bool emit = false;
        if constexpr (BCY == BCY_WALL) {
            if constexpr (cb > 0 && !INTERIOR) emit = ys < 0;
            if constexpr (cb < 0 && !INTERIOR) emit = ys >= p.ny;
        } else {
            if constexpr (cb > 0) ys = ys < 0 ? ys + p.ny : ys;
            if constexpr (cb < 0) ys = ys >= p.ny ? ys - p.ny : ys;
        }
        if (emit) {
            constexpr int side = cb > 0 ? 0 : 1;
            const float rwb = rw[side] * (float)kRest<LY>.w[b];
            unroll<L::QX>([&](auto A) {
                constexpr int a = A;
                if constexpr (L::shifted)
                    v[b][a] = __builtin_fmaf(rwb, p.fw[side][a], -kShift<LX, LY>.s[b][a]);
                else
                    v[b][a] = rwb * p.fw[side][a];
            });
        } else {
            const uint32_t rowb = row_bytes<L::EB>(p, ys);
            unroll<L::QX>([&](auto A) {
                constexpr int a = A;
                v[b][a] = ld<ST>(rs, xa.template src<a>(rowb), (uint32_t)(b * L::QX + a) * p.plane_bytes);
            });
        }
    });
}

// Populations of one node in registers, one FP32 value each: the velocity
// rows b >= B0 of the node, row b in v[b - B0] (all rows by default).
template <int LX, int LY, int B0 = 0, int NB = Axis<LY>::Q>
struct FloatRegs {
    float (&v)[NB][Axis<LX>::Q];
    template <int b, int a>
    __device__ __forceinline__ float get() const { return v[b - B0][a]; }
    template <int b, int a>
    __device__ __forceinline__ void put(float x) { v[b - B0][a] = x; }
};

// Populations of one node in registers as BF16 pairs (two per 32-bit
// register, population q in half q % 2 of register q / 2): half the register
// footprint of FloatRegs, so twice the waves per SIMD.  put() rounds as the
// storage does, so the stores are exact.  With B0 > 0 the registers hold the
// velocity rows from B0 on (q counted from row B0; the random bits of the
// stochastic rounding stay those of the population's own index).
template <int LX, int LY, int ST, int B0 = 0, int NPW = (Axis<LX>::Q * Axis<LY>::Q + 1) / 2>
struct PackedRegs {
    static constexpr int QX = Axis<LX>::Q, NP = NPW;
    uint32_t (&pk)[NP];
    uint32_t h;  // node hash for the stochastic rounding
    template <int b, int a>
    __device__ __forceinline__ float get() const
    {
        constexpr int ql = (b - B0) * QX + a;
        const uint32_t w = pk[ql >> 1];
        return __builtin_bit_cast(float, (ql & 1) ? (w & 0xffff0000u) : (w << 16));
    }
    template <int b, int a>
    __device__ __forceinline__ void put(float x)
    {
        constexpr int q = b * QX + a, ql = (b - B0) * QX + a;
        if constexpr (ST == ST_BF16SR) {
            bf16x2_t hv = __builtin_bit_cast(bf16x2_t, pk[ql >> 1]);
            hv = __builtin_amdgcn_cvt_sr_bf16_f32(hv, x, rnd_of<q>(h), (ql & 1) != 0);
            pk[ql >> 1] = __builtin_bit_cast(uint32_t, hv);
        } else {
            const uint32_t bits = __builtin_bit_cast(unsigned short, (__bf16)x);
            pk[ql >> 1] = (ql & 1) ? ((pk[ql >> 1] & 0xffffu) | (bits << 16)) : ((pk[ql >> 1] & 0xffff0000u) | bits);
        }
    }
};

// Lattices whose nodes the interior-row step splits over two waves (more
// than 144 velocities: a whole node does not fit two waves' registers): the
// first wave of a pair holds the velocity rows b < split_row, the second the
// others, and the two exchange their partial moment sums.
template <int LX, int LY, int ST>
constexpr bool split_node()
{
    return Lat<LX, LY, ST>::Q > 144;
}
template <int LY>
constexpr int split_row()
{
    return (Axis<LY>::Q + 1) / 2;
}

// Mass and momentum sums of the working values of velocity rows [B0, B1).
template <int LX, int LY, int ST, int B0, int B1, class Regs>
__device__ __forceinline__ void moment_sums(const Regs &v, float &r, float &jx, float &jy)
{
    r = 0.0f;
    jx = 0.0f;
    jy = 0.0f;
    unroll_from<B0, B1>([&](auto B) {
        constexpr int b = B, cb = Axis<LY>::c(b);
        float rs = 0.0f, rx = 0.0f;
        unroll<Axis<LX>::Q>([&](auto A) {
            constexpr int a = A, ca = Axis<LX>::c(a);
            const float f = v.template get<b, a>();
            rs += f;
            if constexpr (ca != 0) rx = __builtin_fmaf((float)ca, f, rx);
        });
        r += rs;
        jx += rx;
        if constexpr (cb != 0) jy = __builtin_fmaf((float)cb, rs, jy);
    });
}

// Density and velocity from the sums (the shift has unit mass and no
// momentum).
template <int LX, int LY, int ST>
__device__ __forceinline__ void finish_moments(float r, float jx, float jy, float &rho, float &ux, float &uy)
{
    rho = Lat<LX, LY, ST>::shifted ? kShift<LX, LY>.sum + r : r;
    const float inv = 1.0f / rho;
    ux = jx * inv;
    uy = jy * inv;
}

// Density, momentum and velocity from working values.  Split lattices sum
// the two halves of the velocity rows separately and then add them, as the
// two waves of the split step do, so that every path gives the same bits.
template <int LX, int LY, int ST, class Regs>
__device__ __forceinline__ void density_velocity(const Regs &v, float &rho, float &jx, float &jy, float &ux, float &uy)
{
    float r;
    if constexpr (split_node<LX, LY, ST>()) {
        constexpr int H = split_row<LY>();
        float r0, x0, y0, r1, x1, y1;
        moment_sums<LX, LY, ST, 0, H>(v, r0, x0, y0);
        moment_sums<LX, LY, ST, H, Axis<LY>::Q>(v, r1, x1, y1);
        r = r0 + r1;
        jx = x0 + x1;
        jy = y0 + y1;
    } else {
        moment_sums<LX, LY, ST, 0, Axis<LY>::Q>(v, r, jx, jy);
    }
    finish_moments<LX, LY, ST>(r, jx, jy, rho, ux, uy);
}

// Storages whose update draws random bits: stochastic rounding of the BF16
// stores, and the dithered FP32 update below.
template <int ST>
constexpr bool draws_bits()
{
    return ST == ST_BF16SR || ST == ST_F32S;
}

// f + omega neq + force, rounded once.  FP32 deviation storage rounds the sum
// without bias: a dither uniform over one unit in the last place of the sum
// (from the exponent of the sum rounded to nearest, and 32 random bits) is
// added to the increment, so that the rounding to nearest of f + increment +
// dither rounds f + increment up or down with the probabilities of its
// position between the two neighbours.  Without it, increments below half a
// unit of f are lost every step, and at a small collision frequency the
// steady state sits about eps |f| / (2 omega) from the exact one.  (The
// dither's scale is taken from the sum, which the collision produces late,
// rather than from f: formed from f, the scheduler computed all Q dithers
// next to the loads and ran out of registers.)  Other storages: plain fused
// multiply-adds.  The force enters as gk * w (its shape per axis).
template <int ST, int q>
__device__ __forceinline__ float relax_update(float f, float om, float neq, float gk, float w, uint32_t h)
{
    if constexpr (ST == ST_F32S) {
        const float inc = __builtin_fmaf(om, neq, gk * w);
        const int e = __builtin_amdgcn_frexp_expf(f + inc);  // f + inc = m 2^e, 1/2 <= |m| < 1
        // the population's random word from the node's, mixed with the
        // increment's bits before the rotation: still uniform, and nothing of
        // it can be formed before the collision
        const uint32_t rnd = rnd_of<q>(h ^ __builtin_bit_cast(uint32_t, inc));
        const float d = __builtin_ldexpf((float)(int32_t)rnd, e - 56);  // uniform in [-ulp/2, ulp/2)
        return f + (inc + d);
    } else {
        return __builtin_fmaf(gk, w, __builtin_fmaf(om, neq, f));
    }
}

// BGK collision with the linear force, in place on working values:
// f* = f + omega (rho F_a(u_x) F_b(u_y) - f) + W_a W_b c_a g / theta_x.
// The relaxation is written as f + omega (f^eq - f) so that no rounded
// 1 - omega enters.  In exact arithmetic f^eq carries the mass and momentum
// of f; the FP32 tables rho F_a and F_b do so only up to their rounding,
// deterministically in u, which a channel flow (u constant along rows) would
// integrate into a drift over thousands of steps.  The exact (FP64) sums of
// the FP32 tables give that defect, and it is taken out of the equilibrium of
// the slowest populations (mass: the rest population, or the symmetric set of
// smallest |c| on axes without one) and of the c = +-1 populations among them
// (momentum).
template <int LX, int LY, int ST, int B0 = 0, int B1 = Axis<LY>::Q, class Regs>
__device__ __forceinline__ void collide(const KArgs &p, Regs &v, float rho, float jx, float jy, float ux, float uy,
                                        uint32_t h)
{
    using L = Lat<LX, LY, ST>;
    // per-axis equilibrium in FP64 (the FP64 FMA rate equals the unpacked FP32
    // rate on this chip), each entry then rounded once to FP32
    const float om = p.omega;
    float rF[L::QX], gK[L::QX], Fy[L::QY];
    double sx = 0.0, mx = 0.0, sy = 0.0, my = 0.0;
    {
        double Fd[L::QX];
        axis_equilibrium<LX, double>((double)ux, Fd);
        unroll<L::QX>([&](auto A) {
            constexpr int a = A, ca = Axis<LX>::c(a);
            rF[a] = (float)((double)rho * Fd[a]);
            sx += (double)rF[a];
            mx += (double)ca * (double)rF[a];
            gK[a] = p.gth * (float)(kRest<LX>.w[a] * ca);
        });
    }
    {
        double Fd[L::QY];
        axis_equilibrium<LY, double>((double)uy, Fd);
        unroll<L::QY>([&](auto B) {
            constexpr int b = B, cb = Axis<LY>::c(b);
            Fy[b] = (float)Fd[b];
            sy += (double)Fy[b];
            my += (double)cb * (double)Fy[b];
        });
    }
    // sum f^eq = sx sy, sum f^eq c_x = mx sy, sum f^eq c_y = sx my (exactly, for
    // the products of the FP32 tables)
    // spread over the mx (my) populations of smallest |c_x| (|c_y|): powers of
    // two, so the shares are exact
    constexpr int nx_min = Axis<LX>::cmin ? 2 : 1, ny_min = Axis<LY>::cmin ? 2 : 1;
    const float dm = (float)(sx * sy - (double)rho) * (1.0f / (nx_min * ny_min));
    const float hx = (float)(0.5 * (mx * sy - (double)jx)) * (1.0f / ny_min);
    const float hy = (float)(0.5 * (sx * my - (double)jy)) * (1.0f / nx_min);
    // relax the rows [B0, B1) held (all of them unless the node is split)
    unroll_from<B0, B1>([&](auto B) {
        constexpr int b = B, cb = Axis<LY>::c(b);
        constexpr bool ymin = (cb < 0 ? -cb : cb) == Axis<LY>::cmin;
        unroll<L::QX>([&](auto A) {
            constexpr int a = A, ca = Axis<LX>::c(a);
            constexpr bool xmin = (ca < 0 ? -ca : ca) == Axis<LX>::cmin;
            const float f = v.template get<b, a>();
            float neq;  // f^eq - f
            if constexpr (L::shifted)
                neq = __builtin_fmaf(rF[a], Fy[b], -kShift<LX, LY>.s[b][a]) - f;
            else
                neq = __builtin_fmaf(rF[a], Fy[b], -f);
            if constexpr (xmin && ymin) neq -= dm;
            if constexpr (ymin && ca == 1) neq -= hx;
            if constexpr (ymin && ca == -1) neq += hx;
            if constexpr (xmin && cb == 1) neq -= hy;
            if constexpr (xmin && cb == -1) neq += hy;
            v.template put<b, a>(relax_update<ST, b * L::QX + a>(f, om, neq, gK[a], (float)kRest<LY>.w[b], h));
        });
    });
}

// Store working values at node x of row y, replicating edge nodes into the
// ghost columns when x is periodic.  `h` seeds the stochastic rounding.
template <int LX, int LY, int ST, int BCX>
__device__ __forceinline__ void store_node(const KArgs &p, rsrc_t rd, int x, int y,
                                           const float (&v)[Axis<LY>::Q][Axis<LX>::Q], uint32_t h)
{
    using L = Lat<LX, LY, ST>;
    constexpr int V = Axis<LX>::vmax;
    // columns holding node x: its own, and with periodic padded rows every
    // column of [G - V, G + nx + V) congruent to it modulo nx
    int pc = x + kGhost;
    if constexpr (BCX == BCX_WRAP) pc = x;
    if constexpr (BCX == BCX_PERIODIC) pc = kGhost - V + (x + V) % p.nx;
    for (; pc < kGhost + p.nx + V; pc += p.nx) {
        const uint32_t off = (uint32_t)(y * p.nxp + pc) * (uint32_t)L::EB;
        unroll<L::QY>([&](auto B) {
            unroll<L::QX>([&](auto A) {
                constexpr int a = A, b = B;
                uint32_t r = 0;
                if constexpr (ST == ST_BF16SR) r = rnd_of<b * L::QX + a>(h);
                st<ST>(rd, off, (uint32_t)(b * L::QX + a) * p.plane_bytes, v[b][a], r);
            });
        });
        if constexpr (BCX != BCX_PERIODIC) break;
    }
}

// Hash of (node, step) for the stochastic rounding: reproducible, independent
// of the launch shape.
__device__ __forceinline__ uint32_t node_hash(uint32_t seed, int i)
{
    return mix32((uint32_t)i ^ seed);
}

// Random bits of a node for its storage: BF16 stochastic rounding keys them
// by the node index; the FP32 dither by the row y alone (the same across x and
// z), so that a lattice uniform across x (and z) stays bitwise uniform, as it
// does without random bits.
template <int ST>
__device__ __forceinline__ uint32_t storage_hash(uint32_t seed, int i, int y)
{
    if constexpr (ST == ST_BF16SR) return node_hash(seed, i);
    if constexpr (ST == ST_F32S) return node_hash(seed, y);
    return 0u;
}

// Seed of the stochastic rounding for the step that produces time t (host and
// device: a batched lattice draws the same bits as the lattice alone): a
// golden-ratio Weyl step followed by the first two xor-shift-multiply rounds
// of the splitmix64 finaliser (Steele, Lea and Flood, 2014).
__host__ __device__ inline uint32_t step_seed(int64_t t)
{
    uint64_t x = (uint64_t)t * 0x9e3779b97f4a7c15ULL + 0x632be59bd9b4e019ULL;
    x ^= x >> 31;
    x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 29;
    return (uint32_t)(x >> 32);
}

// An empty register constraint on every word: afterwards the compiler must
// treat the words as changed (no instruction is emitted), so values derived
// from them earlier are recomputed instead of kept live.
template <int Q>
__device__ __forceinline__ void opaque_words(uint32_t (&w)[Q])
{
#pragma unroll
    for (int i = 0; i < Q; ++i) asm volatile("" : "+v"(w[i]));
}

// ------------------------------------------------------------- kernels
// One step of a node with 16-bit storage that takes no wall emission: the
// populations stay packed two per register from the loads to the stores.
template <int LX, int LY, int ST, int BCX, int BCY>
__device__ __forceinline__ void step_packed(const KArgs &p, rsrc_t rs, rsrc_t rd, int x, int y, uint32_t h)
{
    using L = Lat<LX, LY, ST>;
    using P = PackedRegs<LX, LY, ST>;
    const XAddr<LX, 2, BCX> xa(x, p.nx);
    uint32_t pk[P::NP];
    unroll<L::QY>([&](auto B) {
        constexpr int b = B, cb = Axis<LY>::c(b);
        int ys = y - cb;
        if constexpr (BCY != BCY_WALL) {
            if constexpr (cb > 0) ys = ys < 0 ? ys + p.ny : ys;
            if constexpr (cb < 0) ys = ys >= p.ny ? ys - p.ny : ys;
        }
        const uint32_t rowb = row_bytes<2>(p, ys);
        unroll<L::QX>([&](auto A) {
            constexpr int a = A, q = b * L::QX + a;
            const uint32_t raw = (uint32_t)__builtin_bit_cast(
                unsigned short,
                __builtin_amdgcn_raw_buffer_load_b16(rs, xa.template src_lane<a>(rowb),
                                                     (uint32_t)q * p.plane_bytes + decltype(xa)::template src_uniform<a>(), 0));
            if constexpr ((q & 1) == 0)
                pk[q >> 1] = raw;
            else
                pk[q >> 1] |= raw << 16;
        });
    });
    P regs{pk, h};
    float rho, jx, jy, ux, uy;
    density_velocity<LX, LY, ST>(regs, rho, jx, jy, ux, uy);
    // With stochastic rounding, unpack again in the collision: holding all Q
    // unpacked values beside the packed words (the compiler's choice) pushed
    // the kernel into spills or accumulation registers (2.3-3.1x slower at 196
    // and 225 velocities).  Round to nearest is faster left alone.
    if constexpr (ST == ST_BF16SR) opaque_words(pk);
    collide<LX, LY, ST>(p, regs, rho, jx, jy, ux, uy, h);
    constexpr int V = Axis<LX>::vmax;
    int pc = x + kGhost;
    if constexpr (BCX == BCX_WRAP) pc = x;
    if constexpr (BCX == BCX_PERIODIC) pc = kGhost - V + (x + V) % p.nx;
    for (; pc < kGhost + p.nx + V; pc += p.nx) {
        const uint32_t off = (uint32_t)(y * p.nxp + pc) * 2u;
        unroll<L::Q>([&](auto Qi) {
            constexpr int q = Qi;
            const unsigned short half = (q & 1) ? (unsigned short)(pk[q >> 1] >> 16) : (unsigned short)pk[q >> 1];
            __builtin_amdgcn_raw_buffer_store_b16(half, rd, off, (uint32_t)q * p.plane_bytes, kStoreNT);
        });
        if constexpr (BCX != BCX_PERIODIC) break;
    }
}

// Rows a step launch covers: all of them, the rows that take no wall
// emission, or the rows next to each wall that take it (as many as the
// fastest y velocity reaches).
enum StepRows { ROWS_ALL = 0, ROWS_INTERIOR = 1, ROWS_WALLS = 2 };

// One time step of node i: pull from f*(t-1), collide, write f*(t).  With
// 16-bit storage the populations stay packed in registers (PackedRegs)
// wherever no wall emission enters (ROWS_INTERIOR); the wall rows of such a
// lattice are a separate launch (ROWS_WALLS, FP32 registers, so that emitted
// populations enter the collision unrounded), which keeps the packed
// kernel's register allocation its own.
// PRE: wall factors from the wall pre-pass (single-lattice launches of the
// lattices with wall_prepass).
template <int LX, int LY, int ST, int BCX, int BCY, int ROWS, bool PRE = false>
__device__ __forceinline__ void step_node(const KArgs &p, int i, uint32_t seed)
{
    using L = Lat<LX, LY, ST>;
    const int y = i / p.nx, x = i - y * p.nx;
    const rsrc_t rs = make_rsrc(p.src, p.buf_bytes);
    const rsrc_t rd = make_rsrc(p.dst, p.buf_bytes);
    const uint32_t h = storage_hash<ST>(seed, i, y);
    if constexpr (L::EB == 2 && ROWS == ROWS_INTERIOR) {
        step_packed<LX, LY, ST, BCX, BCY>(p, rs, rd, x, y, h);
    } else {
        float v[L::QY][L::QX];
        const XAddr<LX, L::EB, BCX> xa(x, p.nx);
        pull<LX, LY, ST, BCX, BCY, ROWS == ROWS_INTERIOR, PRE>(p, rs, xa, x, y, v);
        FloatRegs<LX, LY> regs{v};
        float rho, jx, jy, ux, uy;
        density_velocity<LX, LY, ST>(regs, rho, jx, jy, ux, uy);
        collide<LX, LY, ST>(p, regs, rho, jx, jy, ux, uy, mix32(h));
        store_node<LX, LY, ST, BCX>(p, rd, x, y, v, h);
    }
}

// Node index of launch index i for a set of rows (see StepRows); -1 outside.
template <int LY, int ROWS>
__device__ __forceinline__ int row_set_node(int i, int nx, int ny)
{
    constexpr int R = Axis<LY>::vmax;
    if constexpr (ROWS == ROWS_ALL) {
        return i < nx * ny ? i : -1;
    } else if constexpr (ROWS == ROWS_INTERIOR) {
        return i < (ny - 2 * R) * nx ? i + R * nx : -1;
    } else {
        if (i >= 2 * R * nx) return -1;
        return i < R * nx ? i : i + (ny - 2 * R) * nx;
    }
}

// ------------------------------------------------ the split interior step
// The nodes of a split lattice (split_node) in compact rows, all of them
// with a periodic y, the interior rows with walls: a block of 256 lanes steps
// 128 nodes, each by a pair of its waves (waves 2g and 2g + 1
// for the 64 nodes of group g), the first holding the velocity rows [0, H),
// the second [H, QY), H = split_row.  Each wave pulls, sums, relaxes and
// stores only its rows, so a node's populations take half the registers and
// twice the waves fit.  The partial sums of mass and momentum meet in LDS
// and are added in the order density_velocity adds them (first half plus
// second half): the node's arithmetic is bitwise that of the unsplit node
// code, which the batched and wall-row launches run.
constexpr int kSplitNodes = kBlock / 2;

// Row that velocity row b of row y pulls from: y - c_b, wrapped across a
// periodic y (the rows reached stay within one period); with walls the split
// step takes only interior rows, whose sources lie inside.
template <int LY, int BCY, int cb>
__device__ __forceinline__ int source_row(int y, int ny)
{
    int ys = y - cb;
    if constexpr (BCY == BCY_PERIODIC) {
        if constexpr (cb > 0) ys = ys < 0 ? ys + ny : ys;
        if constexpr (cb < 0) ys = ys >= ny ? ys - ny : ys;
    }
    return ys;
}

// Words of [B0, B1) packed two per register, counted from row B0.
template <int LX, int LY, int BCX, int BCY, int B0, int B1, int NP>
__device__ __forceinline__ void load_packed_rows(const KArgs &p, rsrc_t rs, const XAddr<LX, 2, BCX> &xa, int y,
                                                 uint32_t (&pk)[NP])
{
    constexpr int QX = Axis<LX>::Q;
    unroll_from<B0, B1>([&](auto B) {
        constexpr int b = B, cb = Axis<LY>::c(b);
        const uint32_t rowb = row_bytes<2>(p, source_row<LY, BCY, cb>(y, p.ny));
        unroll<QX>([&](auto A) {
            constexpr int a = A, q = b * QX + a, ql = (b - B0) * QX + a;
            const uint32_t raw = (uint32_t)__builtin_bit_cast(
                unsigned short,
                __builtin_amdgcn_raw_buffer_load_b16(rs, xa.template src_lane<a>(rowb),
                                                     (uint32_t)q * p.plane_bytes + XAddr<LX, 2, BCX>::template src_uniform<a>(), 0));
            if constexpr ((ql & 1) == 0)
                pk[ql >> 1] = raw;
            else
                pk[ql >> 1] |= raw << 16;
        });
    });
}

template <int LX, int LY, int B0, int B1, int NP>
__device__ __forceinline__ void store_packed_rows(const KArgs &p, rsrc_t rd, uint32_t off, const uint32_t (&pk)[NP])
{
    constexpr int QX = Axis<LX>::Q;
    unroll<(B1 - B0) * QX>([&](auto Ql) {
        constexpr int ql = Ql, q = B0 * QX + ql;
        const unsigned short half = (ql & 1) ? (unsigned short)(pk[ql >> 1] >> 16) : (unsigned short)pk[ql >> 1];
        __builtin_amdgcn_raw_buffer_store_b16(half, rd, off, (uint32_t)q * p.plane_bytes, kStoreNT);
    });
}

// FP32 working values of rows [B0, B1) in v[b - B0] (no wall emission: a
// periodic y, or the interior rows of a channel).
template <int LX, int LY, int ST, int BCX, int BCY, int B0, int B1, int NB>
__device__ __forceinline__ void pull_rows(const KArgs &p, rsrc_t rs, const XAddr<LX, Elem<ST>::bytes, BCX> &xa, int y,
                                          float (&v)[NB][Axis<LX>::Q])
{
    constexpr int QX = Axis<LX>::Q, EB = Elem<ST>::bytes;
    unroll_from<B0, B1>([&](auto B) {
        constexpr int b = B, cb = Axis<LY>::c(b);
        const uint32_t rowb = row_bytes<EB>(p, source_row<LY, BCY, cb>(y, p.ny));
        unroll<QX>([&](auto A) {
            constexpr int a = A;
            v[b - B0][a] = ld<ST>(rs, xa.template src<a>(rowb), (uint32_t)(b * QX + a) * p.plane_bytes);
        });
    });
}

template <int LX, int LY, int ST, int B0, int B1, int NB>
__device__ __forceinline__ void store_rows(const KArgs &p, rsrc_t rd, uint32_t off, const float (&v)[NB][Axis<LX>::Q])
{
    constexpr int QX = Axis<LX>::Q;
    unroll_from<B0, B1>([&](auto B) {
        unroll<QX>([&](auto A) {
            constexpr int a = A, b = B;
            st<ST>(rd, off, (uint32_t)(b * QX + a) * p.plane_bytes, v[b - B0][a]);
        });
    });
}

// The first N words of w opaque to the compiler (see opaque_words).
template <int N, int NP>
__device__ __forceinline__ void opaque_first(uint32_t (&w)[NP])
{
#pragma unroll
    for (int i = 0; i < N; ++i) asm volatile("" : "+v"(w[i]));
}

// Waves per SIMD asked of the register allocator by the single-lattice step
// kernel: two for FP32 storages up to 121 velocities, which fit 256
// registers without spills (left alone, the allocator took 256 registers and
// accumulation registers for the dithered update at 121 velocities: one wave
// per SIMD, 18% slower); no request beyond, or for the 16-bit wall-row
// launches.  (The same request spilled in the resident and three-dimensional
// kernels, which are left alone.)
template <int LX, int LY, int ST, int ROWS = ROWS_ALL>
constexpr int step_waves()
{
    return Elem<ST>::bytes == 4 && Lat<LX, LY, ST>::Q <= 121 && ROWS != ROWS_WALLS ? 2 : 1;
}

// Whether the FP32 rows kernel also steps the wall rows (in its first
// blocks): where the wall path fits its two-wave register budget, i.e. walls
// reaching up to 25 rows; at 27 rows (the G-D1Q28 axis) the absorbed-mass
// sums spilled, and the wall rows get a launch of their own.
template <int LY>
constexpr bool fp32_merged_walls()
{
    return Axis<LY>::vmax <= 25;
}

template <int LX, int LY, int ST, int BCX, int BCY, int ROWS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(step_waves<LX, LY, ST, ROWS>()))) void
step_kernel(KArgs p)
{
    const int i = row_set_node<LY, ROWS>(tile_index(p) * kBlock + (int)threadIdx.x, p.nx, p.ny);
    if (i < 0) return;
    step_node<LX, LY, ST, BCX, BCY, ROWS, BCY == BCY_WALL && wall_prepass<LX, LY, ST>()>(p, i, p.seed);
}

// Wall pre-pass of a single-lattice step with walls (wall_prepass): the
// bottom and top wall factors of every column into p.wrate ([nx] each).  A
// block takes kBlock / 2 columns, its first two waves the bottom wall and the
// other two the top one.
template <int LX, int LY, int ST, int BCX>
__global__ __launch_bounds__(kBlock) void wall_rate_kernel(KArgs p)
{
    const int x = blockIdx.x * (kBlock / 2) + ((int)threadIdx.x & (kBlock / 2 - 1));
    const bool top = (int)threadIdx.x >= kBlock / 2;
    if (x >= p.nx) return;
    const rsrc_t rs = make_rsrc(p.src, p.buf_bytes);
    const XAddr<LX, Elem<ST>::bytes, BCX> xa(x, p.nx);
    if (top)
        p.wrate[p.nx + x] = wall_factor<LX, LY, ST, BCX, false>(p, rs, xa);
    else
        p.wrate[x] = wall_factor<LX, LY, ST, BCX, true>(p, rs, xa);
}

// Blocks of the wall rows in a merged 16-bit launch (a multiple of 8).
template <int LY>
__host__ __device__ constexpr int wall_blocks(int nx)
{
    return ((2 * Axis<LY>::vmax * nx + kBlock - 1) / kBlock + 7) / 8 * 8;
}

// Whether the 16-bit interior and wall rows share one launch: where the wall
// rows' FP32 registers fit beside the packed kernel's budget (two waves up to
// 121 velocities; one wave beyond 144); at 144 velocities the wall path
// needs more than two waves allow.
template <int LX, int LY, int ST>
constexpr bool merged_walls()
{
    return Lat<LX, LY, ST>::Q <= 121 || Lat<LX, LY, ST>::Q > 144;
}

// Waves per SIMD to ask of the register allocator for the 16-bit kernels: two
// up to 144 velocities; beyond, two waves would force large spills (the
// populations of a node do not fit 256 registers beside the collision), so
// the allocator is left free (one wave, no spills).
template <int LX, int LY, int ST>
constexpr int packed_waves()
{
    return Lat<LX, LY, ST>::Q <= 144 ? 2 : 1;
}

// Waves per SIMD asked of the register allocator by the rows kernel: the
// packed 16-bit budget; two for FP32 up to 121 velocities (the dithered
// update took the G-D2Q(12x12) rows kernel to one wave otherwise; at 144
// velocities two waves spill), none beyond.
template <int LX, int LY, int ST>
constexpr int interior_waves()
{
    return Elem<ST>::bytes == 2 ? packed_waves<LX, LY, ST>() : (Lat<LX, LY, ST>::Q <= 121 ? 2 : 1);
}

// The interior rows of a lattice with walls (no wall emission reaches them:
// a pull without branches), in FP32 registers or, with 16-bit storage,
// packed two per register.  For the packed rows the register allocator is
// asked for two waves per SIMD up to 144 velocities: left to itself the
// scheduler sinks the packing of loaded pairs to their use (hiding load
// latency) and ends a few registers above the 256 that two waves allow,
// halving the bytes in flight of a memory-bound kernel.
//
// WALLS: the same launch also steps the rows next to the walls (FP32
// registers), in its first blocks (a multiple of 8, so that the interior
// blocks keep their XCD order): the small, latency-bound wall rows then run
// beside the interior instead of in a launch of their own after it.
template <int LX, int LY, int ST, int BCX, int BCY, bool WALLS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(interior_waves<LX, LY, ST>()))) void
step_kernel_rows(KArgs p)
{
    int b = blockIdx.x, G = gridDim.x;
    if constexpr (WALLS) {
        const int wb = wall_blocks<LY>(p.nx);
        if (b < wb) {
            const int i = row_set_node<LY, ROWS_WALLS>(b * kBlock + (int)threadIdx.x, p.nx, p.ny);
            if (i >= 0) step_node<LX, LY, ST, BCX, BCY, ROWS_WALLS, wall_prepass<LX, LY, ST>()>(p, i, p.seed);
            return;
        }
        b -= wb;
        G -= wb;
    }
    const int i = row_set_node<LY, ROWS_INTERIOR>(tile_of(b, G, p.remap) * kBlock + (int)threadIdx.x, p.nx, p.ny);
    if (i < 0) return;
    step_node<LX, LY, ST, BCX, BCY, ROWS_INTERIOR>(p, i, p.seed);
}

// Nodes of a split lattice over wave pairs (see kSplitNodes): every node
// with a periodic y; the interior rows with walls, whose wall rows are a
// launch of their own (one node per lane in FP32 registers with the wall
// sums: in the same kernel they would set its register budget).  Two waves
// per SIMD are asked of the register allocator.
template <int LX, int LY, int ST, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void step_kernel_split(KArgs p)
{
    static_assert(BCX == BCX_WRAP, "the split step is built for compact rows");
    using L = Lat<LX, LY, ST>;
    constexpr int QX = L::QX, QY = L::QY, H = split_row<LY>(), R = Axis<LY>::vmax;
    constexpr int ROWS = BCY == BCY_WALL ? ROWS_INTERIOR : ROWS_ALL;
    __shared__ float xch[kBlock / 64][3][64];
    const int b = blockIdx.x, G = gridDim.x;
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63, half = wave & 1;
    const int in = row_set_node<LY, ROWS>(tile_of(b, G, p.remap) * kSplitNodes + (wave >> 1) * 64 + lane, p.nx, p.ny);
    // lanes past the last node step the first node of the row set and store
    // nothing (every wave must reach the barrier)
    const bool valid = in >= 0;
    const int i = valid ? in : (BCY == BCY_WALL ? R * p.nx : 0);
    const int y = i / p.nx, x = i - y * p.nx;
    const rsrc_t rs = make_rsrc(p.src, p.buf_bytes);
    const rsrc_t rd = make_rsrc(p.dst, p.buf_bytes);
    const uint32_t h = storage_hash<ST>(p.seed, i, y);
    const XAddr<LX, L::EB, BCX> xa(x, p.nx);
    const uint32_t off = (uint32_t)(y * p.nxp + x) * (uint32_t)L::EB;
    float r, jx, jy;
    auto exchange = [&](float &R0, float &JX, float &JY) {
        xch[wave][0][lane] = r;
        xch[wave][1][lane] = jx;
        xch[wave][2][lane] = jy;
        __syncthreads();
        const int w0 = wave & ~1, w1 = w0 | 1;  // first half + second half
        R0 = xch[w0][0][lane] + xch[w1][0][lane];
        JX = xch[w0][1][lane] + xch[w1][1][lane];
        JY = xch[w0][2][lane] + xch[w1][2][lane];
    };
    float R0, JX, JY, rho, ux, uy;
    if constexpr (L::EB == 2) {
        constexpr int NP = (H * QX + 1) / 2;  // the larger half
        uint32_t pk[NP];
        if (half == 0) {
            load_packed_rows<LX, LY, BCX, BCY, 0, H>(p, rs, xa, y, pk);
            moment_sums<LX, LY, ST, 0, H>(PackedRegs<LX, LY, ST, 0, NP>{pk, h}, r, jx, jy);
        } else {
            load_packed_rows<LX, LY, BCX, BCY, H, QY>(p, rs, xa, y, pk);
            moment_sums<LX, LY, ST, H, QY>(PackedRegs<LX, LY, ST, H, NP>{pk, h}, r, jx, jy);
        }
        exchange(R0, JX, JY);
        finish_moments<LX, LY, ST>(R0, JX, JY, rho, ux, uy);
        if (half == 0) {
            if constexpr (ST == ST_BF16SR) opaque_first<(H * QX + 1) / 2>(pk);
            PackedRegs<LX, LY, ST, 0, NP> regs{pk, h};
            collide<LX, LY, ST, 0, H>(p, regs, rho, JX, JY, ux, uy, h);
            if (valid) store_packed_rows<LX, LY, 0, H>(p, rd, off, pk);
        } else {
            if constexpr (ST == ST_BF16SR) opaque_first<((QY - H) * QX + 1) / 2>(pk);
            PackedRegs<LX, LY, ST, H, NP> regs{pk, h};
            collide<LX, LY, ST, H, QY>(p, regs, rho, JX, JY, ux, uy, h);
            if (valid) store_packed_rows<LX, LY, H, QY>(p, rd, off, pk);
        }
    } else {
        float v[H][QX];
        if (half == 0) {
            pull_rows<LX, LY, ST, BCX, BCY, 0, H>(p, rs, xa, y, v);
            moment_sums<LX, LY, ST, 0, H>(FloatRegs<LX, LY, 0, H>{v}, r, jx, jy);
        } else {
            pull_rows<LX, LY, ST, BCX, BCY, H, QY>(p, rs, xa, y, v);
            moment_sums<LX, LY, ST, H, QY>(FloatRegs<LX, LY, H, H>{v}, r, jx, jy);
        }
        exchange(R0, JX, JY);
        finish_moments<LX, LY, ST>(R0, JX, JY, rho, ux, uy);
        if (half == 0) {
            FloatRegs<LX, LY, 0, H> regs{v};
            collide<LX, LY, ST, 0, H>(p, regs, rho, JX, JY, ux, uy, mix32(h));
            if (valid) store_rows<LX, LY, ST, 0, H>(p, rd, off, v);
        } else {
            FloatRegs<LX, LY, H, H> regs{v};
            collide<LX, LY, ST, H, QY>(p, regs, rho, JX, JY, ux, uy, mix32(h));
            if (valid) store_rows<LX, LY, ST, H, QY>(p, rd, off, v);
        }
    }
}

// Batched step: many lattices of one variant in one launch.  Block b takes
// tile b = (member, first launch index, count) of the table; the member's
// arguments for this launch's parity are read through the scalar unit, and
// the node runs exactly the single-lattice code, so that a batched lattice is
// bitwise the lattice stepped alone.
struct BatchTile {
    int32_t member, first, count, pad;
};

// Launch `launch` of a chunk: batch step s = *bstep + launch; member m is at
// time t0[m] + s, its f*(t) in buffer phase[m] ^ (s & 1).  args holds two
// argument sets per member, args[2m + c] pulling from buffer c.
template <int LX, int LY, int ST, int BCX, int BCY, int ROWS>
__global__ __launch_bounds__(kBlock) void batch_step_kernel(const BatchTile *__restrict__ tiles,
                                                            const KArgs *__restrict__ args,
                                                            const int32_t *__restrict__ phase,
                                                            const int64_t *__restrict__ t0,
                                                            const int64_t *__restrict__ bstep, int32_t launch)
{
    const BatchTile t = tiles[blockIdx.x];
    if ((int)threadIdx.x >= t.count) return;
    const int64_t s = *bstep + launch;
    const KArgs &p = args[2 * t.member + (phase[t.member] ^ (int)(s & 1))];
    const int i = row_set_node<LY, ROWS>(t.first + (int)threadIdx.x, p.nx, p.ny);
    if (i < 0) return;
    step_node<LX, LY, ST, BCX, BCY, ROWS>(p, i, draws_bits<ST>() ? step_seed(t0[t.member] + s + 1) : 0u);
}

// Resident batched steps for small lattices: block b owns member
// members[b] whole and advances it `steps` steps of a chunk (batch steps
// *bstep .. *bstep + steps - 1), looping over the member's nodes, with a
// workgroup barrier between steps (a step's stores, made by this workgroup
// on this compute unit, are visible to its loads of the next step).  One
// launch per chunk instead of one per step; every node runs the
// single-lattice code with the same seeds, so the result is bitwise the
// lattice stepped alone.  16-bit storage with walls takes its interior rows
// packed and its wall rows in FP32, as the step launches do.
template <int LX, int LY, int ST, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void resident_step_kernel(const int32_t *__restrict__ members,
                                                               const KArgs *__restrict__ args,
                                                               const int32_t *__restrict__ phase,
                                                               const int64_t *__restrict__ t0,
                                                               const int64_t *__restrict__ bstep, int32_t steps)
{
    constexpr bool split = Elem<ST>::bytes == 2 && BCY == BCY_WALL;
    const int m = members[blockIdx.x];
    const int64_t s0 = *bstep;
    const int ph = phase[m];
    const int64_t tm = t0[m];
    for (int l = 0; l < steps; ++l) {
        const int64_t s = s0 + l;
        const KArgs &p = args[2 * m + (ph ^ (int)(s & 1))];
        const uint32_t seed = draws_bits<ST>() ? step_seed(tm + s + 1) : 0u;
        if constexpr (split) {
            constexpr int R = Axis<LY>::vmax;
            const int interior = (p.ny - 2 * R) * p.nx, walls = 2 * R * p.nx;
            for (int j = threadIdx.x; j < interior; j += kBlock)
                step_node<LX, LY, ST, BCX, BCY, ROWS_INTERIOR>(p, row_set_node<LY, ROWS_INTERIOR>(j, p.nx, p.ny), seed);
            for (int j = threadIdx.x; j < walls; j += kBlock)
                step_node<LX, LY, ST, BCX, BCY, ROWS_WALLS>(p, row_set_node<LY, ROWS_WALLS>(j, p.nx, p.ny), seed);
        } else {
            const int n = p.nx * p.ny;
            for (int j = threadIdx.x; j < n; j += kBlock) step_node<LX, LY, ST, BCX, BCY, ROWS_ALL>(p, j, seed);
        }
        __syncthreads();
    }
}

// Moments (and optionally the populations) of the pre-collision state f(t).
// A diagnostics kernel: the stored FP32 values are summed in FP64, so the
// reported moments carry the state's error and no evaluation noise.
template <int LX, int LY, int ST, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void observe_kernel(KArgs p)
{
    using L = Lat<LX, LY, ST>;
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i >= p.nodes) return;
    const int y = i / p.nx, x = i - y * p.nx;
    const rsrc_t rs = make_rsrc(p.src, p.buf_bytes);
    float v[L::QY][L::QX];
    const XAddr<LX, L::EB, BCX> xa(x, p.nx);
    if (p.local) {
        const uint32_t base = xa.own(row_bytes<L::EB>(p, y));
        unroll<L::QY>([&](auto B) {
            unroll<L::QX>([&](auto A) {
                constexpr int a = A, b = B;
                v[b][a] = ld<ST>(rs, base, (uint32_t)(b * L::QX + a) * p.plane_bytes);
            });
        });
    } else {
        pull<LX, LY, ST, BCX, BCY>(p, rs, xa, x, y, v);
    }
    double r = 0.0, jx = 0.0, jy = 0.0;
    unroll<L::QY>([&](auto B) {
        unroll<L::QX>([&](auto A) {
            constexpr int a = A, b = B, ca = Axis<LX>::c(a), cb = Axis<LY>::c(b);
            const double f = v[b][a];
            r += f;
            jx += ca * f;
            jy += cb * f;
        });
    });
    const double rho = L::shifted ? (double)kShift<LX, LY>.sum + r : r;
    const double ux = jx / rho, uy = jy / rho;
    // second moments from f - f^eq: the product equilibrium has
    // sum f^eq c_x^2 = rho (u_x^2 + theta_x) and sum f^eq c_x c_y = rho u_x u_y,
    // so T = (theta_x + theta_y + sum (f - f^eq) |c|^2 / rho) / dims and
    // Pxy = sum (f - f^eq) c_x c_y
    double Fx[L::QX], Fy[L::QY];
    axis_equilibrium<LX, double>(ux, Fx);
    axis_equilibrium<LY, double>(uy, Fy);
    double e2 = 0.0, exy = 0.0;
    unroll<L::QY>([&](auto B) {
        unroll<L::QX>([&](auto A) {
            constexpr int a = A, b = B, ca = Axis<LX>::c(a), cb = Axis<LY>::c(b);
            double f = v[b][a];
            if constexpr (L::shifted) f += (double)kShift<LX, LY>.s[b][a];
            const double dev = f - rho * Fx[a] * Fy[b];
            e2 += (ca * ca + cb * cb) * dev;
            exy += (ca * cb) * dev;
        });
    });
    constexpr int dims = LY > 0 ? 2 : 1;
    if (p.o_rho) p.o_rho[i] = (float)rho;
    if (p.o_ux) p.o_ux[i] = (float)ux;
    if (p.o_uy) p.o_uy[i] = (float)uy;
    if (p.o_T) p.o_T[i] = (float)((Axis<LX>::theta + Axis<LY>::theta + e2 / rho) / dims);
    if (p.o_pxy) p.o_pxy[i] = (float)exy;
    if (p.o_f) {
        unroll<L::QY>([&](auto B) {
            unroll<L::QX>([&](auto A) {
                constexpr int a = A, b = B;
                float f = v[b][a];
                if constexpr (L::shifted) f += kShift<LX, LY>.s[b][a];
                p.o_f[(size_t)(b * L::QX + a) * p.nodes + i] = f;
            });
        });
    }
}

// f(0) from fields (equilibrium) or given populations; writes f(0) into dst2
// and f*(0) = collide(f(0)) into dst.
template <int LX, int LY, int ST, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void init_kernel(KArgs p)
{
    using L = Lat<LX, LY, ST>;
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i >= p.nodes) return;
    const int y = i / p.nx, x = i - y * p.nx;
    float v[L::QY][L::QX];
    if (p.i_f) {
        unroll<L::QY>([&](auto B) {
            unroll<L::QX>([&](auto A) {
                constexpr int a = A, b = B;
                v[b][a] = p.i_f[(size_t)(b * L::QX + a) * p.nodes + i];
            });
        });
    } else {
        const float rho = p.i_rho ? p.i_rho[i] : 1.0f;
        const float ux = p.i_ux ? p.i_ux[i] : 0.0f;
        const float uy = (p.i_uy && LY > 0) ? p.i_uy[i] : 0.0f;
        double Fx[L::QX], Fy[L::QY];
        axis_equilibrium<LX, double>((double)ux, Fx);
        axis_equilibrium<LY, double>((double)uy, Fy);
        unroll<L::QY>([&](auto B) {
            unroll<L::QX>([&](auto A) {
                constexpr int a = A, b = B;
                v[b][a] = (float)((double)rho * Fx[a] * Fy[b]);
            });
        });
    }
    if constexpr (L::shifted) {
        unroll<L::QY>([&](auto B) {
            unroll<L::QX>([&](auto A) {
                constexpr int a = A, b = B;
                v[b][a] -= kShift<LX, LY>.s[b][a];
            });
        });
    }
    const uint32_t h = storage_hash<ST>(p.seed, i, y);
    if constexpr (Elem<ST>::bytes == 2) {
        // round f(0) as the storage will, so that f*(0) is the collision of the
        // stored f(0) (the stores below are then exact)
        unroll<L::QY>([&](auto B) {
            unroll<L::QX>([&](auto A) {
                constexpr int a = A, b = B;
                v[b][a] = quantize<ST>(v[b][a], rnd_of<b * L::QX + a>(h));
            });
        });
    }
    const rsrc_t r2 = make_rsrc(p.dst2, p.buf_bytes);
    store_node<LX, LY, ST, BCX>(p, r2, x, y, v, h);
    FloatRegs<LX, LY> regs{v};
    float rho, jx, jy, ux, uy;
    density_velocity<LX, LY, ST>(regs, rho, jx, jy, ux, uy);
    collide<LX, LY, ST>(p, regs, rho, jx, jy, ux, uy, mix32(mix32(h)));
    const rsrc_t rd = make_rsrc(p.dst, p.buf_bytes);
    store_node<LX, LY, ST, BCX>(p, rd, x, y, v, mix32(h));
}

// Ghost columns of the fixed equilibrium ends: f = rho_end W_a W_b (working
// value minus the shift when shifted), in both buffers.  One thread per
// (q, row, ghost column).
template <int LX, int LY, int ST>
__global__ __launch_bounds__(kBlock) void ends_kernel(KArgs p, float rho_left, float rho_right)
{
    using L = Lat<LX, LY, ST>;
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    constexpr int V = Axis<LX>::vmax;
    const int per_row = 2 * V;
    if (i >= L::Q * p.ny * per_row) return;
    const int q = i / (p.ny * per_row);
    const int rem = i - q * p.ny * per_row;
    const int y = rem / per_row, k = rem - y * per_row;
    const bool left = k < V;
    // k in [0, V): columns G-V .. G-1; k in [V, 2V): columns G+nx .. G+nx+V-1
    const int pc = left ? kGhost - V + k : kGhost + p.nx + (k - V);
    const int a = q % L::QX, b = q / L::QX;
    double w = 1.0, s = 0.0;
    // run-time index into compile-time tables
    unroll<L::QY>([&](auto B) {
        unroll<L::QX>([&](auto A) {
            if (A == a && B == b) {
                w = kRest<LX>.w[A] * kRest<LY>.w[B];
                s = kShift<LX, LY>.s[B][A];
            }
        });
    });
    const double rho = left ? rho_left : rho_right;
    const float val = (float)(L::shifted ? rho * w - s : rho * w);
    const uint32_t off = (uint32_t)(y * p.nxp + pc) * (uint32_t)L::EB;
    // the ends are fixed data, not dynamics: round them to nearest
    constexpr int STN = Elem<ST>::bytes == 2 ? (int)ST_BF16S : ST;
    st<STN>(make_rsrc(p.dst, p.buf_bytes), off, (uint32_t)q * p.plane_bytes, val);
    st<STN>(make_rsrc(p.dst2, p.buf_bytes), off, (uint32_t)q * p.plane_bytes, val);
}

// Global FP64 sums (glbm_stats): per-block partials.
// [0] mass  [1] momentum x  [2] momentum y  [3] energy (post)  [4] sum u_x^2
// [5] sum (u_x(t) - u_x(t-1))^2  [6] bottom absorbed mass  [7] bottom x momentum
// [8] top absorbed mass  [9] top x momentum  [10] nodes outside the positivity
// domain  [11] momentum z (three dimensions)  [12] non-finite nodes
// The blocks stride over the nodes, so that a launch of at most kStatBlocks
// blocks covers any lattice and the partials stay a fixed, small array.
constexpr int kStatBlocks = 2048;

// Failure detection on a node's sums: a density, momentum or energy that is
// not a finite number marks a node that has blown up (it is then not tested
// against the positivity domain).
__device__ __forceinline__ bool finite_node(double r, double jx, double jy, double jz, double e)
{
    return __builtin_isfinite(r) && __builtin_isfinite(jx) && __builtin_isfinite(jy) && __builtin_isfinite(jz) &&
           __builtin_isfinite(e);
}

// Wave reduction of the per-lane sums, then across the block's waves through
// LDS; thread k < kNumStats writes the block's partial k.
__device__ __forceinline__ void write_partials(double (&acc)[kNumStats], double *partials)
{
    __shared__ double red[kBlock / 64][kNumStats];
    for (int k = 0; k < kNumStats; ++k) {
        double s = acc[k];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        acc[k] = s;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < kNumStats; ++k) red[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < kNumStats) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
        partials[(size_t)blockIdx.x * kNumStats + threadIdx.x] = s;
    }
}

template <int LX, int LY, int ST, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void stats_kernel(KArgs p)
{
    using L = Lat<LX, LY, ST>;
    double acc[kNumStats];
    for (int k = 0; k < kNumStats; ++k) acc[k] = 0.0;
    const rsrc_t rs = make_rsrc(p.src, p.buf_bytes);
    for (int i = blockIdx.x * kBlock + (int)threadIdx.x; i < p.nodes; i += gridDim.x * kBlock) {
        const int y = i / p.nx, x = i - y * p.nx;
        const XAddr<LX, L::EB, BCX> xa(x, p.nx);
        const uint32_t base = xa.own(row_bytes<L::EB>(p, y));
        double r = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
        unroll<L::QY>([&](auto B) {
            unroll<L::QX>([&](auto A) {
                constexpr int a = A, b = B, ca = Axis<LX>::c(a), cb = Axis<LY>::c(b);
                const double f = ld<ST>(rs, base, (uint32_t)(b * L::QX + a) * p.plane_bytes);
                r += f;
                jx += ca * f;
                jy += cb * f;
                e += (ca * ca + cb * cb) * f;
            });
        });
        if constexpr (L::shifted) {
            r += (double)kShift<LX, LY>.sum;
            e += (double)kShift<LX, LY>.sxx + (double)kShift<LX, LY>.syy;
        }
        // f*(t) carries the force momentum g of step t's collision
        const double jx_pre = jx - p.g;
        const double ux = jx_pre / r, uy = jy / r;
        acc[0] += r;
        acc[1] += jx_pre;
        acc[2] += jy;
        acc[3] += e;
        acc[4] += ux * ux;
        if (p.prev) {
            const rsrc_t rp = make_rsrc(p.prev, p.buf_bytes);
            double r0 = 0.0, j0 = 0.0;
            unroll<L::QY>([&](auto B) {
                unroll<L::QX>([&](auto A) {
                    constexpr int a = A, b = B, ca = Axis<LX>::c(a);
                    const double f = ld<ST>(rp, base, (uint32_t)(b * L::QX + a) * p.plane_bytes);
                    r0 += f;
                    j0 += ca * f;
                });
            });
            if constexpr (L::shifted) r0 += (double)kShift<LX, LY>.sum;
            const double d = ux - (j0 - p.g) / r0;
            acc[5] += d * d;
        }
        if (!finite_node(r, jx, jy, 0.0, e))
            acc[12] += 1.0;
        else if (ux * ux > Axis<LX>::u2max || (LY > 0 && uy * uy > Axis<LY>::u2max))  // section 3 (Axis::u2max)
            acc[10] += 1.0;
        if constexpr (BCY == BCY_WALL) {
            if (y == 0) {
                float m;
                const float A = wall_absorbed<LX, LY, ST, BCX, true>(p, rs, xa, &m);
                acc[6] += A;
                acc[7] += (double)m - (double)A * p.uw[0];
            }
            if (y == p.ny - 1) {
                float m;
                const float A = wall_absorbed<LX, LY, ST, BCX, false>(p, rs, xa, &m);
                acc[8] += A;
                acc[9] += (double)m - (double)A * p.uw[1];
            }
        }
    }
    write_partials(acc, p.partials);
}

}  // namespace glbm
