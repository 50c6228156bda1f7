// Three-dimensional lattices: the tensor product of three axes (section 4,
// f^eq = rho F_a(u_x) F_b(u_y) F_c(u_z)), periodic in x and z, periodic or
// diffuse walls across y (the reading of sections 5.3-5.4 with the wall
// density per (x, z) column).
//
// Layout: velocity planes [q][z][y][row], q = (c QY + b) QX + a; a row is the
// padded or compact x row of the two-dimensional lattices (XAddr), rows are
// numbered z ny + y.  One lane owns one node and holds its Q populations in
// FP32 registers (every storage); the node's steps are those of the 2D
// kernels with a third factor in the equilibrium, the force shape, the wall
// emission and the mass / momentum defect correction.
#pragma once

#include "glbm_device.h"

namespace glbm {

template <int LX, int LY, int LZ, int ST>
struct Lat3 {
    static constexpr int QX = Axis<LX>::Q, QY = Axis<LY>::Q, QZ = Axis<LZ>::Q, Q = QX * QY * QZ;
    static constexpr int EB = Elem<ST>::bytes;
    static constexpr bool shifted = Elem<ST>::shifted;
    template <int a, int b, int c>
    static constexpr int q() { return (c * QY + b) * QX + a; }
};

// Shift of the shifted storages in three dimensions: S_abc ~ W_a W_b W_c on
// the 2^-24 grid, the remainder shared equally by the slowest populations
// (as ShiftTable), and the moments of S the kernels add back.
template <int LX, int LY, int LZ>
struct ShiftTable3 {
    static constexpr int QX = Axis<LX>::Q, QY = Axis<LY>::Q, QZ = Axis<LZ>::Q;
    float s[QZ][QY][QX];
    float sum, sxx, syy, szz;
    float absorbed;  // sum of S over the populations one wall absorbs per column
    constexpr ShiftTable3() : s{}, sum(0.0f), sxx(0.0f), syy(0.0f), szz(0.0f), absorbed(0.0f)
    {
        long long q[QZ][QY][QX] = {};
        long long tot = 0;
        for (int c = 0; c < QZ; ++c)
            for (int b = 0; b < QY; ++b)
                for (int a = 0; a < QX; ++a)
                    tot += (q[c][b][a] = snap(kRest<LX>.w[a] * kRest<LY>.w[b] * kRest<LZ>.w[c]));
        const long long m = (Axis<LX>::even ? 2 : 1) * (Axis<LY>::even ? 2 : 1) * (Axis<LZ>::even ? 2 : 1);
        const long long rem = (long long)kGrid - tot;
        const long long share = rem >= 0 ? rem / m : -((-rem + m - 1) / m);
        long long all = 0, xx = 0, yy = 0, zz = 0, ab = 0;
        for (int c = 0; c < QZ; ++c)
            for (int b = 0; b < QY; ++b)
                for (int a = 0; a < QX; ++a) {
                    const long long ca = Axis<LX>::c(a), cb = Axis<LY>::c(b), cc = Axis<LZ>::c(c);
                    if ((ca < 0 ? -ca : ca) == Axis<LX>::cmin && (cb < 0 ? -cb : cb) == Axis<LY>::cmin &&
                        (cc < 0 ? -cc : cc) == Axis<LZ>::cmin)
                        q[c][b][a] += share;
                    all += q[c][b][a];
                    xx += q[c][b][a] * ca * ca;
                    yy += q[c][b][a] * cb * cb;
                    zz += q[c][b][a] * cc * cc;
                    if (cb < 0) ab += q[c][b][a] * (-cb);
                    s[c][b][a] = (float)(q[c][b][a] / kGrid);
                }
        sum = (float)(all / kGrid);
        sxx = (float)(xx / kGrid);
        syy = (float)(yy / kGrid);
        szz = (float)(zz / kGrid);
        absorbed = (float)(ab / kGrid);
    }
};

template <int LX, int LY, int LZ>
inline constexpr ShiftTable3<LX, LY, LZ> kShift3{};

// Rest weights of the (y, z) pair in FP32, and the half flux of the y axis
// weighted by them: the wall emits rho_w fw_a W_bc into |c_b| rows, i.e.
// rho_w * sum_a fw_a * J3 per column.
template <int LY, int LZ>
struct YZWeights {
    float w[Axis<LZ>::Q][Axis<LY>::Q];
    double jplus;
    constexpr YZWeights() : w{}, jplus(0.0)
    {
        for (int c = 0; c < Axis<LZ>::Q; ++c)
            for (int b = 0; b < Axis<LY>::Q; ++b) {
                w[c][b] = (float)(kRest<LY>.w[b] * kRest<LZ>.w[c]);
                if (Axis<LY>::c(b) > 0) jplus += Axis<LY>::c(b) * (double)w[c][b];
            }
    }
};

template <int LY, int LZ>
inline constexpr YZWeights<LY, LZ> kYZ{};

template <int LZ>
__device__ __forceinline__ int wrap_z(int zs, int nz)
{
    // nz >= the fastest z velocity: one correction at most
    return zs < 0 ? zs + nz : zs >= nz ? zs - nz : zs;
}

// Mass absorbed by a diffuse wall in column (x, z): the post-collision
// populations leaving through the wall in this streaming that would land in
// (x, z) (sources at x - c_x, z - c_z in the rows within reach).
template <int LX, int LY, int LZ, int ST, int BCX, bool BOTTOM>
__device__ __forceinline__ float wall_absorbed3(const KArgs &p, rsrc_t rs, const XAddr<LX, Elem<ST>::bytes, BCX> &xa,
                                                int z, float *mom)
{
    using L = Lat3<LX, LY, LZ, ST>;
    float s = 0.0f, m = 0.0f;
    unroll<L::QZ>([&](auto C) {
        constexpr int c = C, cc = Axis<LZ>::c(c);
        const int zs = wrap_z<LZ>(z - cc, p.nz);
        unroll<L::QY>([&](auto B) {
            constexpr int b = B, cb = Axis<LY>::c(b);
            if constexpr ((BOTTOM && cb < 0) || (!BOTTOM && cb > 0)) {
                constexpr int depth = cb < 0 ? -cb : cb;
                unroll<depth>([&](auto R) {
                    const int row = BOTTOM ? (int)R : p.ny - 1 - (int)R;
                    const uint32_t rowb = row_bytes<L::EB>(p, zs * p.ny + row);
                    unroll<L::QX>([&](auto A) {
                        constexpr int a = A, ca = Axis<LX>::c(a);
                        const float v = ld<ST>(rs, xa.template src<a>(rowb), (uint32_t)L::template q<a, b, c>() * p.plane_bytes);
                        s += v;
                        if (mom) m = __builtin_fmaf((float)ca, v, m);
                    });
                });
            }
        });
    });
    if (mom) *mom = m;
    if constexpr (L::shifted) s += kShift3<LX, LY, LZ>.absorbed;
    return s;
}

// Wall re-emission factor of the column at (x, z): rho_w / (J+ sum_a fw_a),
// rho_w the mass the wall absorbs there in this streaming.
template <int LX, int LY, int LZ, int ST, int BCX, bool BOTTOM>
__device__ __forceinline__ float wall_factor3(const KArgs &p, rsrc_t rs, const XAddr<LX, Elem<ST>::bytes, BCX> &xa, int z)
{
    constexpr double jp = kYZ<LY, LZ>.jplus;
    return wall_absorbed3<LX, LY, LZ, ST, BCX, BOTTOM>(p, rs, xa, z, nullptr) / (float)(jp * p.fwsum[BOTTOM ? 0 : 1]);
}

// Wall factors of a node in row y for the bottom and top walls (zero out of
// their reach; INTERIOR: none).  PRE: read from the wall pre-pass of this
// step (wall_rate3_kernel, the same arithmetic once per column) instead of
// summed by the lane: every one of the 2 R wall rows of a column would
// otherwise repeat the column's sum (R (R + 1) / 2 rows of QX QZ loads).
template <int LX, int LY, int LZ, int ST, int BCX, int BCY, bool INTERIOR, bool PRE = false>
__device__ __forceinline__ void wall_rates3(const KArgs &p, rsrc_t rs, const XAddr<LX, Elem<ST>::bytes, BCX> &xa, int x,
                                            int y, int z, float (&rw)[2])
{
    rw[0] = 0.0f;
    rw[1] = 0.0f;
    if constexpr (BCY == BCY_WALL && !INTERIOR) {
        constexpr int reach = Axis<LY>::vmax;
        if constexpr (PRE) {
            const int col = z * p.nx + x;
            if (y < reach) rw[0] = p.wrate[col];
            if (y >= p.ny - reach) rw[1] = p.wrate[p.nx * p.nz + col];
        } else {
            if (y < reach) rw[0] = wall_factor3<LX, LY, LZ, ST, BCX, true>(p, rs, xa, z);
            if (y >= p.ny - reach) rw[1] = wall_factor3<LX, LY, LZ, ST, BCX, false>(p, rs, xa, z);
        }
    }
}

// Pre-collision populations of velocity row (b, c) of node (x, y, z):
// pulled, or emitted by a wall (rw from wall_rates3).  INTERIOR: the node is
// at least the fastest y velocity away from both walls, so nothing is emitted
// into it and the pull has no branches (all its loads can be in flight
// together).
template <int LX, int LY, int LZ, int ST, int BCX, int BCY, bool INTERIOR, int b, int c>
__device__ __forceinline__ void pull3_row(const KArgs &p, rsrc_t rs, const XAddr<LX, Elem<ST>::bytes, BCX> &xa, int y,
                                          int z, const float (&rw)[2], float (&row)[Axis<LX>::Q])
{
    using L = Lat3<LX, LY, LZ, ST>;
    constexpr int cb = Axis<LY>::c(b), cc = Axis<LZ>::c(c);
    const int zs = wrap_z<LZ>(z - cc, p.nz);
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
        const float rwb = rw[side] * kYZ<LY, LZ>.w[c][b];
        unroll<L::QX>([&](auto A) {
            constexpr int a = A;
            if constexpr (L::shifted)
                row[a] = __builtin_fmaf(rwb, p.fw[side][a], -kShift3<LX, LY, LZ>.s[c][b][a]);
            else
                row[a] = rwb * p.fw[side][a];
        });
    } else {
        const uint32_t rowb = row_bytes<L::EB>(p, zs * p.ny + ys);
        unroll<L::QX>([&](auto A) {
            constexpr int a = A;
            row[a] = ld<ST>(rs, xa.template src<a>(rowb), (uint32_t)L::template q<a, b, c>() * p.plane_bytes);
        });
    }
}

// Pre-collision populations of node (x, y, z): pulled, or emitted by a wall.
template <int LX, int LY, int LZ, int ST, int BCX, int BCY, bool INTERIOR = false, bool PRE = false>
__device__ __forceinline__ void pull3(const KArgs &p, rsrc_t rs, const XAddr<LX, Elem<ST>::bytes, BCX> &xa, int x, int y,
                                      int z, float (&v)[Axis<LZ>::Q][Axis<LY>::Q][Axis<LX>::Q])
{
    float rw[2];
    wall_rates3<LX, LY, LZ, ST, BCX, BCY, INTERIOR, PRE>(p, rs, xa, x, y, z, rw);
    unroll<Axis<LZ>::Q>([&](auto C) {
        unroll<Axis<LY>::Q>([&](auto B) {
            pull3_row<LX, LY, LZ, ST, BCX, BCY, INTERIOR, (int)B, (int)C>(p, rs, xa, y, z, rw, v[C][B]);
        });
    });
}

// Equilibrium factors of a collision: rho F_a(u_x) and the force shape per x
// velocity, F_b(u_y) F_c(u_z) of the velocity rows [R0, R1) (row r = c QY + b),
// and the conservative defect correction: the FP32 tables rho F_a and F_b F_c
// carry the mass and momentum only up to rounding; the exact (FP64) sums over
// every row give the defect, which the slowest populations take out.
template <int LX, int LY, int LZ, int R0, int R1>
struct Eq3 {
    float rF[Axis<LX>::Q], gK[Axis<LX>::Q], FYZ[R1 - R0];
    float dm, hx, hy, hz;
};

// The per-axis FP64 equilibrium tables of a node: F_a(u_x), F_b(u_y), F_c(u_z)
// at unit density.
template <int LX, int LY, int LZ>
__device__ __forceinline__ void eq3_tables(float ux, float uy, float uz, double (&Fx)[Axis<LX>::Q],
                                           double (&Fy)[Axis<LY>::Q], double (&Fz)[Axis<LZ>::Q])
{
    axis_equilibrium<LX, double>((double)ux, Fx);
    axis_equilibrium<LY, double>((double)uy, Fy);
    axis_equilibrium<LZ, double>((double)uz, Fz);
}

// The defect corrections dm, hx, hy, hz from the tables: the mass and
// momentum that the FP32 factors rho F_a and F_b F_c miss, summed in FP64
// over every row.
template <int LX, int LY, int LZ, class TX, class TY, class TZ>
__device__ __forceinline__ void eq3_defects(float rho, float jx, float jy, float jz, const TX &Fx, const TY &Fy,
                                            const TZ &Fz, float (&d)[4])
{
    constexpr int QX = Axis<LX>::Q, QY = Axis<LY>::Q, QZ = Axis<LZ>::Q;
    double sx = 0.0, mx = 0.0, syz = 0.0, my = 0.0, mz = 0.0;
    unroll<QX>([&](auto A) {
        constexpr int a = A, ca = Axis<LX>::c(a);
        const float rF = (float)((double)rho * Fx(a));
        sx += (double)rF;
        mx += (double)ca * (double)rF;
    });
    unroll<QZ>([&](auto C) {
        constexpr int c = C, cc = Axis<LZ>::c(c);
        unroll<QY>([&](auto B) {
            constexpr int b = B, cb = Axis<LY>::c(b);
            const float fyz = (float)(Fy(b) * Fz(c));
            syz += (double)fyz;
            my += (double)cb * (double)fyz;
            mz += (double)cc * (double)fyz;
        });
    });
    constexpr int nxm = Axis<LX>::cmin ? 2 : 1, nym = Axis<LY>::cmin ? 2 : 1, nzm = Axis<LZ>::cmin ? 2 : 1;
    d[0] = (float)(sx * syz - (double)rho) * (1.0f / (nxm * nym * nzm));
    d[1] = (float)(0.5 * (mx * syz - (double)jx)) * (1.0f / (nym * nzm));
    d[2] = (float)(0.5 * (sx * my - (double)jy)) * (1.0f / (nxm * nzm));
    d[3] = (float)(0.5 * (sx * mz - (double)jz)) * (1.0f / (nxm * nym));
}

// The FP32 factors of the rows [R0, R1) from the tables.
template <int LX, int LY, int LZ, int R0, int R1, class TX, class TY, class TZ>
__device__ __forceinline__ void eq3_rows(const KArgs &p, float rho, const TX &Fx, const TY &Fy, const TZ &Fz,
                                         Eq3<LX, LY, LZ, R0, R1> &e)
{
    constexpr int QX = Axis<LX>::Q, QY = Axis<LY>::Q;
    unroll<QX>([&](auto A) {
        constexpr int a = A, ca = Axis<LX>::c(a);
        e.rF[a] = (float)((double)rho * Fx(a));
        e.gK[a] = p.gth * (float)(kRest<LX>.w[a] * ca);
    });
    unroll_from<R0, R1>([&](auto Rr) {
        constexpr int r = Rr, c = r / QY, b = r % QY;
        e.FYZ[r - R0] = (float)(Fy(b) * Fz(c));
    });
}

// All factors of a collision of the rows [R0, R1) (one lane computes the whole
// node's tables and defects).
template <int LX, int LY, int LZ, int R0, int R1>
__device__ __forceinline__ void eq3_factors(const KArgs &p, float rho, float jx, float jy, float jz, float ux, float uy,
                                            float uz, Eq3<LX, LY, LZ, R0, R1> &e)
{
    double Fx[Axis<LX>::Q], Fy[Axis<LY>::Q], Fz[Axis<LZ>::Q];
    eq3_tables<LX, LY, LZ>(ux, uy, uz, Fx, Fy, Fz);
    auto fx = [&](int a) { return Fx[a]; };
    auto fy = [&](int b) { return Fy[b]; };
    auto fz = [&](int c) { return Fz[c]; };
    float d[4];
    eq3_defects<LX, LY, LZ>(rho, jx, jy, jz, fx, fy, fz, d);
    e.dm = d[0];
    e.hx = d[1];
    e.hy = d[2];
    e.hz = d[3];
    eq3_rows<LX, LY, LZ, R0, R1>(p, rho, fx, fy, fz, e);
}

// BGK relaxation with the linear force (section 5.4) of the velocity rows
// [R0, R1); at(r, a) is the FP32 working value of population (a, row r).
template <int LX, int LY, int LZ, int ST, int R0, int R1, class At>
__device__ __forceinline__ void relax3_rows(const KArgs &p, const Eq3<LX, LY, LZ, R0, R1> &e, At &&at, uint32_t h)
{
    using L = Lat3<LX, LY, LZ, ST>;
    const float om = p.omega;
    unroll_from<R0, R1>([&](auto Rr) {
        constexpr int r = Rr, c = r / L::QY, b = r % L::QY, cc = Axis<LZ>::c(c), cb = Axis<LY>::c(b);
        constexpr bool zmin = (cc < 0 ? -cc : cc) == Axis<LZ>::cmin;
        constexpr bool ymin = (cb < 0 ? -cb : cb) == Axis<LY>::cmin;
        unroll<L::QX>([&](auto A) {
            constexpr int a = A, ca = Axis<LX>::c(a);
            constexpr bool xmin = (ca < 0 ? -ca : ca) == Axis<LX>::cmin;
            float &v = at(Rr, A);
            const float f = v;
            float neq;  // f^eq - f
            if constexpr (L::shifted)
                neq = __builtin_fmaf(e.rF[a], e.FYZ[r - R0], -kShift3<LX, LY, LZ>.s[c][b][a]) - f;
            else
                neq = __builtin_fmaf(e.rF[a], e.FYZ[r - R0], -f);
            if constexpr (xmin && ymin && zmin) neq -= e.dm;
            if constexpr (ymin && zmin && ca == 1) neq -= e.hx;
            if constexpr (ymin && zmin && ca == -1) neq += e.hx;
            if constexpr (xmin && zmin && cb == 1) neq -= e.hy;
            if constexpr (xmin && zmin && cb == -1) neq += e.hy;
            if constexpr (xmin && ymin && cc == 1) neq -= e.hz;
            if constexpr (xmin && ymin && cc == -1) neq += e.hz;
            v = relax_update<ST, L::template q<a, b, c>()>(f, om, neq, e.gK[a], kYZ<LY, LZ>.w[c][b], h);
        });
    });
}

// Collision of a whole node.
template <int LX, int LY, int LZ, int ST>
__device__ __forceinline__ void collide3(const KArgs &p, float (&v)[Axis<LZ>::Q][Axis<LY>::Q][Axis<LX>::Q], float rho,
                                         float jx, float jy, float jz, float ux, float uy, float uz, uint32_t h)
{
    constexpr int QY = Axis<LY>::Q, NR = Axis<LZ>::Q * QY;
    Eq3<LX, LY, LZ, 0, NR> e;
    eq3_factors<LX, LY, LZ, 0, NR>(p, rho, jx, jy, jz, ux, uy, uz, e);
    relax3_rows<LX, LY, LZ, ST, 0, NR>(
        p, e,
        [&](auto Rr, auto A) -> float & {
            constexpr int r = Rr, a = A;
            return v[r / QY][r % QY][a];
        },
        h);
}

template <int LX, int LY, int LZ, int ST>
__device__ __forceinline__ void moments3(const float (&v)[Axis<LZ>::Q][Axis<LY>::Q][Axis<LX>::Q], float &rho, float &jx,
                                         float &jy, float &jz)
{
    using L = Lat3<LX, LY, LZ, ST>;
    float r = 0.0f;
    jx = jy = jz = 0.0f;
    unroll<L::QZ>([&](auto C) {
        constexpr int c = C, cc = Axis<LZ>::c(c);
        float rc = 0.0f;
        unroll<L::QY>([&](auto B) {
            constexpr int b = B, cb = Axis<LY>::c(b);
            float rs = 0.0f, rx = 0.0f;
            unroll<L::QX>([&](auto A) {
                constexpr int a = A, ca = Axis<LX>::c(a);
                rs += v[c][b][a];
                if constexpr (ca != 0) rx = __builtin_fmaf((float)ca, v[c][b][a], rx);
            });
            rc += rs;
            jx += rx;
            if constexpr (cb != 0) jy = __builtin_fmaf((float)cb, rs, jy);
        });
        r += rc;
        if constexpr (cc != 0) jz = __builtin_fmaf((float)cc, rc, jz);
    });
    rho = L::shifted ? kShift3<LX, LY, LZ>.sum + r : r;
}

// Store node (x, y, z), replicating edge nodes into the ghost columns of
// padded periodic rows.
template <int LX, int LY, int LZ, int ST, int BCX>
__device__ __forceinline__ void store3(const KArgs &p, rsrc_t rd, int x, int row,
                                       const float (&v)[Axis<LZ>::Q][Axis<LY>::Q][Axis<LX>::Q], uint32_t h)
{
    using L = Lat3<LX, LY, LZ, ST>;
    constexpr int V = Axis<LX>::vmax;
    int pc = x + kGhost;
    if constexpr (BCX == BCX_WRAP) pc = x;
    if constexpr (BCX == BCX_PERIODIC) pc = kGhost - V + (x + V) % p.nx;
    for (; pc < kGhost + p.nx + V; pc += p.nx) {
        const uint32_t off = (uint32_t)(row * p.nxp + pc) * (uint32_t)L::EB;
        unroll<L::QZ>([&](auto C) {
            unroll<L::QY>([&](auto B) {
                unroll<L::QX>([&](auto A) {
                    constexpr int a = A, b = B, c = C, q = L::template q<a, b, c>();
                    uint32_t r = 0;
                    if constexpr (ST == ST_BF16SR) r = rnd_of<q>(h);
                    st<ST>(rd, off, (uint32_t)q * p.plane_bytes, v[c][b][a], r);
                });
            });
        });
        if constexpr (BCX != BCX_PERIODIC) break;
    }
}

__device__ __forceinline__ void node_xyz(const KArgs &p, int i, int &x, int &y, int &z)
{
    const int r = i / p.nx;
    x = i - r * p.nx;
    z = r / p.ny;
    y = r - z * p.ny;
}

// Blocks of the wall rows of a 3D step with walls, nb nodes per block (a
// multiple of 8).
template <int LY>
__host__ __device__ constexpr int wall_blocks3(int nx, int nz, int nb)
{
    return ((2 * Axis<LY>::vmax * nx * nz + nb - 1) / nb + 7) / 8 * 8;
}

// ------------------------------------------- nodes split over waves
// Above 125 velocities a node's populations and the collision do not fit one
// lane's registers at two waves per SIMD (at 126-144 the compiler spilled to
// accumulation registers and ran one wave; the 343 of G-D3Q343 do not fit at
// all), so the step splits each node over split3_waves waves of a block:
// two from 100 velocities on in FP32 (neutral there: the step is
// memory-bound) and from 64 on in 16-bit storage (whose step is VALU-bound:
// three waves per SIMD instead of two, 0.48-0.52 -> 0.55-0.59 of 8 TB/s at
// 108-125 velocities; at 126-144 two waves per node beat four, 0.45-0.49 ->
// 0.49-0.56); four above 144:
// wave g holds the velocity rows [split3_row(g), split3_row(g + 1)) of its
// nodes (row r = c QY + b, QX populations each), pulls, sums, relaxes and
// stores only those; the partial sums of mass and momentum meet in LDS and
// are added in wave order.  The first wave of each node's group then forms
// the node's FP64 axis tables and defect corrections, shared through LDS
// behind a second barrier (formed by every wave they were a third of the
// VALU work of a 16-bit split step, which is VALU-bound), and each wave its
// rows' FP32 factors from them.  The one-lane node code (the batched step)
// adds the same partial sums in the same order and forms the same tables,
// so a node gives the same bits split or not.
template <int LX, int LY, int LZ, int ST>
constexpr int split3_waves()
{
    constexpr int Q = Lat3<LX, LY, LZ, ST>::Q;
    if constexpr (Elem<ST>::bytes == 2) return Q > 144 ? 4 : Q > 63 ? 2 : 1;
    return Q > 144 ? 4 : Q > 99 ? 2 : 1;
}
template <int LX, int LY, int LZ, int ST>
constexpr bool split3()
{
    return split3_waves<LX, LY, LZ, ST>() > 1;
}
template <int LY, int LZ, int K>
__host__ __device__ constexpr int split3_row(int g)
{
    return (Axis<LY>::Q * Axis<LZ>::Q * g + K - 1) / K;
}

// Mass and momentum sums of the velocity rows [R0, R1) (working values).
template <int LX, int LY, int LZ, int R0, int R1, class At>
__device__ __forceinline__ void moments3_rows(At &&at, float &r, float &jx, float &jy, float &jz)
{
    r = jx = jy = jz = 0.0f;
    unroll_from<R0, R1>([&](auto Rr) {
        constexpr int rr = Rr, c = rr / Axis<LY>::Q, b = rr % Axis<LY>::Q;
        constexpr int cb = Axis<LY>::c(b), cc = Axis<LZ>::c(c);
        float rs = 0.0f, rx = 0.0f;
        unroll<Axis<LX>::Q>([&](auto A) {
            constexpr int ca = Axis<LX>::c((int)A);
            const float f = at(Rr, A);
            rs += f;
            if constexpr (ca != 0) rx = __builtin_fmaf((float)ca, f, rx);
        });
        r += rs;
        jx += rx;
        if constexpr (cb != 0) jy = __builtin_fmaf((float)cb, rs, jy);
        if constexpr (cc != 0) jz = __builtin_fmaf((float)cc, rs, jz);
    });
}

// Mass and momentum of a whole node in registers: for a split lattice the
// partial sums of its wave parts, added in wave order (as the split step).
template <int LX, int LY, int LZ, int ST>
__device__ __forceinline__ void node_moments3(const float (&v)[Axis<LZ>::Q][Axis<LY>::Q][Axis<LX>::Q], float &rho,
                                              float &jx, float &jy, float &jz)
{
    using L = Lat3<LX, LY, LZ, ST>;
    constexpr int K = split3_waves<LX, LY, LZ, ST>();
    if constexpr (K == 1) {
        moments3<LX, LY, LZ, ST>(v, rho, jx, jy, jz);
    } else {
        float m[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        unroll<K>([&](auto G) {
            constexpr int R0 = split3_row<LY, LZ, K>(G), R1 = split3_row<LY, LZ, K>(G + 1);
            float q[4];
            moments3_rows<LX, LY, LZ, R0, R1>(
                [&](auto Rr, auto A) -> float { return v[(int)Rr / L::QY][(int)Rr % L::QY][(int)A]; }, q[0], q[1], q[2],
                q[3]);
            for (int k = 0; k < 4; ++k) m[k] = G == 0 ? q[k] : m[k] + q[k];
        });
        rho = L::shifted ? kShift3<LX, LY, LZ>.sum + m[0] : m[0];
        jx = m[1];
        jy = m[2];
        jz = m[3];
    }
}

// One node (x, y, z) of a step with the random-bit seed of that step;
// INTERIOR: no wall emission reaches it; PRE: wall factors from the wall
// pre-pass.
template <int LX, int LY, int LZ, int ST, int BCX, int BCY, bool INTERIOR, bool PRE = false>
__device__ __forceinline__ void step3_node(const KArgs &p, int x, int y, int z, uint32_t seed)
{
    using L = Lat3<LX, LY, LZ, ST>;
    const int i = (z * p.ny + y) * p.nx + x;
    const rsrc_t rs = make_rsrc(p.src, p.buf_bytes);
    const rsrc_t rd = make_rsrc(p.dst, p.buf_bytes);
    const XAddr<LX, L::EB, BCX> xa(x, p.nx);
    float v[L::QZ][L::QY][L::QX];
    pull3<LX, LY, LZ, ST, BCX, BCY, INTERIOR, PRE>(p, rs, xa, x, y, z, v);
    float rho, jx, jy, jz;
    node_moments3<LX, LY, LZ, ST>(v, rho, jx, jy, jz);
    const float inv = 1.0f / rho;
    const uint32_t h = storage_hash<ST>(seed, i, y);
    collide3<LX, LY, LZ, ST>(p, v, rho, jx, jy, jz, jx * inv, jy * inv, jz * inv, mix32(h));
    store3<LX, LY, LZ, ST, BCX>(p, rd, x, z * p.ny + y, v, h);
}

// Node of launch index j within a set of rows of every z plane: the rows
// that take no wall emission, or the rows next to the walls (as many as the
// fastest y velocity reaches); false outside the set.
template <int LY, int ROWS>
__device__ __forceinline__ bool row_set_node3(const KArgs &p, int j, int &x, int &y, int &z)
{
    constexpr int R = Axis<LY>::vmax;
    const int rows = ROWS == ROWS_INTERIOR ? p.ny - 2 * R : 2 * R;
    const int per = rows * p.nx;
    if (j >= per * p.nz) return false;
    z = j / per;
    const int r = j - z * per;
    const int yr = r / p.nx;
    x = r - yr * p.nx;
    y = ROWS == ROWS_INTERIOR ? yr + R : (yr < R ? yr : p.ny - 2 * R + yr);
    return true;
}

// Wall pre-pass of a step with walls: the bottom and top wall factors of
// every (x, z) column into p.wrate (the wall rows of the step then read them
// instead of each summing its column).  A block takes kBlock / 2 columns,
// its first two waves the bottom wall and the other two the top one.
template <int LX, int LY, int LZ, int ST, int BCX>
__global__ __launch_bounds__(kBlock) void wall_rate3_kernel(KArgs p)
{
    const int col = blockIdx.x * (kBlock / 2) + ((int)threadIdx.x & (kBlock / 2 - 1));
    const bool top = (int)threadIdx.x >= kBlock / 2;
    if (col >= p.nx * p.nz) return;
    const int z = col / p.nx, x = col - z * p.nx;
    const rsrc_t rs = make_rsrc(p.src, p.buf_bytes);
    const XAddr<LX, Elem<ST>::bytes, BCX> xa(x, p.nx);
    if (top)
        p.wrate[p.nx * p.nz + col] = wall_factor3<LX, LY, LZ, ST, BCX, false>(p, rs, xa, z);
    else
        p.wrate[col] = wall_factor3<LX, LY, LZ, ST, BCX, true>(p, rs, xa, z);
}

// One step.  Periodic y: every node alike.  Walls: one launch whose first
// blocks (a multiple of 8, so that the others keep their XCD order) step the
// rows next to the walls (wall factors from the pre-pass) and the others the
// interior rows, whose pull has no branches (all of a node's loads in flight
// together).  Two waves per SIMD asked of the register allocator (up to 125
// velocities: G-D3Q125 fits 256 registers without spills; left alone, the
// dithered FP32 update took it to one wave).
template <int LX, int LY, int LZ, int ST, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void step3_kernel(KArgs p)
{
    static_assert(!split3<LX, LY, LZ, ST>(), "split lattices step in step3_split_kernel");
    int x, y, z;
    if constexpr (BCY != BCY_WALL) {
        const int j = tile_index(p) * kBlock + (int)threadIdx.x;
        if (j >= p.nodes) return;
        node_xyz(p, j, x, y, z);
        step3_node<LX, LY, LZ, ST, BCX, BCY, false>(p, x, y, z, p.seed);
    } else {
        const int wb = wall_blocks3<LY>(p.nx, p.nz, kBlock);
        const int b = blockIdx.x;
        if (b < wb) {
            if (row_set_node3<LY, ROWS_WALLS>(p, b * kBlock + (int)threadIdx.x, x, y, z))
                step3_node<LX, LY, LZ, ST, BCX, BCY, false, true>(p, x, y, z, p.seed);
            return;
        }
        const int j = tile_of(b - wb, gridDim.x - wb, p.remap) * kBlock + (int)threadIdx.x;
        if (row_set_node3<LY, ROWS_INTERIOR>(p, j, x, y, z)) step3_node<LX, LY, LZ, ST, BCX, BCY, true>(p, x, y, z, p.seed);
    }
}

// Wave g of a split node: its rows of node (x, y, z) pulled and summed into
// the exchange slot of its wave, then (after the block's barrier, which
// every wave reaches once) the node's moments from the K slots of its wave
// group, its rows relaxed and, for a valid node, stored.
// Per-node tables of a split step shared through LDS: the FP64 axis tables
// (QX + QY + QZ entries) and the four defect corrections of each node of
// the block, computed once by the first wave of the node's group.
template <int LX, int LY, int LZ, int NB>
struct SplitTables3 {
    static constexpr int NT = Axis<LX>::Q + Axis<LY>::Q + Axis<LZ>::Q;
    double tab[NT][NB];
    float def[4][NB];
};

template <int LX, int LY, int LZ, int ST, int BCX, int BCY, bool INTERIOR, int NB>
__device__ __forceinline__ void split3_node(const KArgs &p, int g, int x, int y, int z, bool valid,
                                            float (&xch)[kBlock / 64][4][64], SplitTables3<LX, LY, LZ, NB> &sh,
                                            int slot, int wave, int lane)
{
    using L = Lat3<LX, LY, LZ, ST>;
    constexpr int K = split3_waves<LX, LY, LZ, ST>();
    constexpr int QX = L::QX, NR = split3_row<LY, LZ, K>(1);  // the largest part
    static_assert(BCX == BCX_WRAP, "the split step is built for compact rows");
    const int i = (z * p.ny + y) * p.nx + x;
    const rsrc_t rs = make_rsrc(p.src, p.buf_bytes);
    const rsrc_t rd = make_rsrc(p.dst, p.buf_bytes);
    const XAddr<LX, L::EB, BCX> xa(x, p.nx);
    const uint32_t h = storage_hash<ST>(p.seed, i, y);
    float v[NR][QX];
    float rw[2];
    wall_rates3<LX, LY, LZ, ST, BCX, BCY, INTERIOR, true>(p, rs, xa, x, y, z, rw);
    unroll<K>([&](auto G) {
        constexpr int R0 = split3_row<LY, LZ, K>(G), R1 = split3_row<LY, LZ, K>(G + 1);
        if (g == G) {
            unroll_from<R0, R1>([&](auto Rr) {
                constexpr int r = Rr;
                pull3_row<LX, LY, LZ, ST, BCX, BCY, INTERIOR, r % L::QY, r / L::QY>(p, rs, xa, y, z, rw, v[r - R0]);
            });
            float m[4];
            moments3_rows<LX, LY, LZ, R0, R1>([&](auto Rr, auto A) -> float & { return v[(int)Rr - R0][(int)A]; },
                                              m[0], m[1], m[2], m[3]);
            for (int k = 0; k < 4; ++k) xch[wave][k][lane] = m[k];
        }
    });
    __syncthreads();
    const int w0 = wave - g;  // first wave of the group
    float m[4];
    for (int k = 0; k < 4; ++k) {
        m[k] = xch[w0][k][lane];
        for (int j = 1; j < K; ++j) m[k] += xch[w0 + j][k][lane];
    }
    const float rho = L::shifted ? kShift3<LX, LY, LZ>.sum + m[0] : m[0];
    const float inv = 1.0f / rho;
    const uint32_t off = (uint32_t)((z * p.ny + y) * p.nxp + x) * (uint32_t)L::EB;
    // the node's FP64 tables and defects, once per node (the first wave of
    // its group), shared through LDS: the same arithmetic as eq3_factors
    constexpr int QY = L::QY, QZ = L::QZ;
    if (g == 0) {
        double Fx[QX], Fy[QY], Fz[QZ];
        eq3_tables<LX, LY, LZ>(m[1] * inv, m[2] * inv, m[3] * inv, Fx, Fy, Fz);
        float d[4];
        eq3_defects<LX, LY, LZ>(
            rho, m[1], m[2], m[3], [&](int a) { return Fx[a]; }, [&](int b) { return Fy[b]; },
            [&](int c) { return Fz[c]; }, d);
        for (int j = 0; j < QX; ++j) sh.tab[j][slot] = Fx[j];
        for (int j = 0; j < QY; ++j) sh.tab[QX + j][slot] = Fy[j];
        for (int j = 0; j < QZ; ++j) sh.tab[QX + QY + j][slot] = Fz[j];
        for (int k = 0; k < 4; ++k) sh.def[k][slot] = d[k];
    }
    __syncthreads();
    auto fx = [&](int a) { return sh.tab[a][slot]; };
    auto fy = [&](int b) { return sh.tab[QX + b][slot]; };
    auto fz = [&](int c) { return sh.tab[QX + QY + c][slot]; };
    unroll<K>([&](auto G) {
        constexpr int R0 = split3_row<LY, LZ, K>(G), R1 = split3_row<LY, LZ, K>(G + 1);
        if (g == G) {
            auto at = [&](auto Rr, auto A) -> float & { return v[(int)Rr - R0][(int)A]; };
            Eq3<LX, LY, LZ, R0, R1> e;
            eq3_rows<LX, LY, LZ, R0, R1>(p, rho, fx, fy, fz, e);
            e.dm = sh.def[0][slot];
            e.hx = sh.def[1][slot];
            e.hy = sh.def[2][slot];
            e.hz = sh.def[3][slot];
            relax3_rows<LX, LY, LZ, ST, R0, R1>(p, e, at, mix32(h));
            if (valid) {
                unroll_from<R0, R1>([&](auto Rr) {
                    constexpr int r = Rr, c = r / L::QY, b = r % L::QY;
                    unroll<QX>([&](auto A) {
                        constexpr int a = A, q = L::template q<a, b, c>();
                        uint32_t rb = 0;
                        if constexpr (ST == ST_BF16SR) rb = rnd_of<q>(h);
                        st<ST>(rd, off, (uint32_t)q * p.plane_bytes, v[r - R0][a], rb);
                    });
                });
            }
        }
    });
}

// One step of a split lattice: kBlock / K nodes per block, node j of the
// block in lane j % 64 of waves K (j / 64) .. K (j / 64) + K - 1.  Periodic
// y: every node alike.  Walls: the first blocks (a multiple of 8) take the
// rows next to the walls (wall factors from the pre-pass), the others the
// interior rows.  Lanes past the last node step an in-bounds node of their
// set and store nothing (every wave must reach the barrier).  Two waves per
// SIMD asked of the register allocator (three fit at 343 velocities).
template <int LX, int LY, int LZ, int ST, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void step3_split_kernel(KArgs p)
{
    constexpr int K = split3_waves<LX, LY, LZ, ST>(), NB = kBlock / K, R = Axis<LY>::vmax;
    __shared__ float xch[kBlock / 64][4][64];
    __shared__ SplitTables3<LX, LY, LZ, NB> sh;
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63, g = wave % K;
    const int slot = (wave / K) * 64 + lane;
    int x = 0, y = 0, z = 0;
    if constexpr (BCY != BCY_WALL) {
        const int j = tile_index(p) * NB + slot;
        const bool valid = j < p.nodes;
        if (valid) node_xyz(p, j, x, y, z);
        split3_node<LX, LY, LZ, ST, BCX, BCY, false>(p, g, x, y, z, valid, xch, sh, slot, wave, lane);
    } else {
        const int wb = wall_blocks3<LY>(p.nx, p.nz, NB);
        const int b = blockIdx.x;
        if (b < wb) {
            const bool valid = row_set_node3<LY, ROWS_WALLS>(p, b * NB + slot, x, y, z);
            if (!valid) x = y = z = 0;
            split3_node<LX, LY, LZ, ST, BCX, BCY, false>(p, g, x, y, z, valid, xch, sh, slot, wave, lane);
        } else {
            const int j = tile_of(b - wb, gridDim.x - wb, p.remap) * NB + slot;
            const bool valid = row_set_node3<LY, ROWS_INTERIOR>(p, j, x, y, z);
            if (!valid) {
                x = z = 0;
                y = R;
            }
            split3_node<LX, LY, LZ, ST, BCX, BCY, true>(p, g, x, y, z, valid, xch, sh, slot, wave, lane);
        }
    }
}

// Batched step of three-dimensional members (see batch_step_kernel): block
// b takes tile b of the table, nodes first .. first + count - 1 of its
// member in the order (z, y, x), each by the single-lattice node code with
// the pull that checks for wall emission (which loads the same values for an
// interior node): a batched lattice is bitwise the lattice stepped alone.
template <int LX, int LY, int LZ, int ST, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(Lat3<LX, LY, LZ, ST>::Q <= 125 ? 2 : 1))) void
batch_step3_kernel(const BatchTile *__restrict__ tiles, const KArgs *__restrict__ args,
                   const int32_t *__restrict__ phase, const int64_t *__restrict__ t0,
                   const int64_t *__restrict__ bstep, int32_t launch)
{
    const BatchTile t = tiles[blockIdx.x];
    if ((int)threadIdx.x >= t.count) return;
    const int64_t s = *bstep + launch;
    const KArgs &p = args[2 * t.member + (phase[t.member] ^ (int)(s & 1))];
    const int j = t.first + (int)threadIdx.x;
    if (j >= p.nodes) return;
    int x, y, z;
    node_xyz(p, j, x, y, z);
    step3_node<LX, LY, LZ, ST, BCX, BCY, false>(p, x, y, z, draws_bits<ST>() ? step_seed(t0[t.member] + s + 1) : 0u);
}

// Moments of f(t) (FP64 sums of the stored values), as observe_kernel.
template <int LX, int LY, int LZ, int ST, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void observe3_kernel(KArgs p)
{
    using L = Lat3<LX, LY, LZ, ST>;
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i >= p.nodes) return;
    int x, y, z;
    node_xyz(p, i, x, y, z);
    const rsrc_t rs = make_rsrc(p.src, p.buf_bytes);
    const XAddr<LX, L::EB, BCX> xa(x, p.nx);
    float v[L::QZ][L::QY][L::QX];
    if (p.local) {
        const uint32_t base = xa.own(row_bytes<L::EB>(p, z * p.ny + y));
        unroll<L::QZ>([&](auto C) {
            unroll<L::QY>([&](auto B) {
                unroll<L::QX>([&](auto A) {
                    constexpr int a = A, b = B, c = C;
                    v[c][b][a] = ld<ST>(rs, base, (uint32_t)L::template q<a, b, c>() * p.plane_bytes);
                });
            });
        });
    } else {
        pull3<LX, LY, LZ, ST, BCX, BCY>(p, rs, xa, x, y, z, v);
    }
    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    unroll<L::QZ>([&](auto C) {
        unroll<L::QY>([&](auto B) {
            unroll<L::QX>([&](auto A) {
                constexpr int a = A, b = B, c = C;
                const double f = v[c][b][a];
                r += f;
                jx += Axis<LX>::c(a) * f;
                jy += Axis<LY>::c(b) * f;
                jz += Axis<LZ>::c(c) * f;
            });
        });
    });
    const double rho = L::shifted ? (double)kShift3<LX, LY, LZ>.sum + r : r;
    const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
    double Fx[L::QX], Fy[L::QY], Fz[L::QZ];
    axis_equilibrium<LX, double>(ux, Fx);
    axis_equilibrium<LY, double>(uy, Fy);
    axis_equilibrium<LZ, double>(uz, Fz);
    double e2 = 0.0, exy = 0.0;
    unroll<L::QZ>([&](auto C) {
        unroll<L::QY>([&](auto B) {
            unroll<L::QX>([&](auto A) {
                constexpr int a = A, b = B, c = C, ca = Axis<LX>::c(a), cb = Axis<LY>::c(b), cc = Axis<LZ>::c(c);
                double f = v[c][b][a];
                if constexpr (L::shifted) f += (double)kShift3<LX, LY, LZ>.s[c][b][a];
                const double dev = f - rho * Fx[a] * Fy[b] * Fz[c];
                e2 += (ca * ca + cb * cb + cc * cc) * dev;
                exy += (ca * cb) * dev;
            });
        });
    });
    if (p.o_rho) p.o_rho[i] = (float)rho;
    if (p.o_ux) p.o_ux[i] = (float)ux;
    if (p.o_uy) p.o_uy[i] = (float)uy;
    if (p.o_uz) p.o_uz[i] = (float)uz;
    if (p.o_T) p.o_T[i] = (float)((Axis<LX>::theta + Axis<LY>::theta + Axis<LZ>::theta + e2 / rho) / 3.0);
    if (p.o_pxy) p.o_pxy[i] = (float)exy;
    if (p.o_f) {
        unroll<L::QZ>([&](auto C) {
            unroll<L::QY>([&](auto B) {
                unroll<L::QX>([&](auto A) {
                    constexpr int a = A, b = B, c = C;
                    float f = v[c][b][a];
                    if constexpr (L::shifted) f += kShift3<LX, LY, LZ>.s[c][b][a];
                    p.o_f[(size_t)L::template q<a, b, c>() * p.nodes + i] = f;
                });
            });
        });
    }
}

// f(0) from fields or populations into dst2, f*(0) into dst.
template <int LX, int LY, int LZ, int ST, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void init3_kernel(KArgs p)
{
    using L = Lat3<LX, LY, LZ, ST>;
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i >= p.nodes) return;
    int x, y, z;
    node_xyz(p, i, x, y, z);
    float v[L::QZ][L::QY][L::QX];
    if (p.i_f) {
        unroll<L::QZ>([&](auto C) {
            unroll<L::QY>([&](auto B) {
                unroll<L::QX>([&](auto A) {
                    constexpr int a = A, b = B, c = C;
                    v[c][b][a] = p.i_f[(size_t)L::template q<a, b, c>() * p.nodes + i];
                });
            });
        });
    } else {
        const double rho = p.i_rho ? p.i_rho[i] : 1.0;
        double Fx[L::QX], Fy[L::QY], Fz[L::QZ];
        axis_equilibrium<LX, double>(p.i_ux ? (double)p.i_ux[i] : 0.0, Fx);
        axis_equilibrium<LY, double>(p.i_uy ? (double)p.i_uy[i] : 0.0, Fy);
        axis_equilibrium<LZ, double>(p.i_uz ? (double)p.i_uz[i] : 0.0, Fz);
        unroll<L::QZ>([&](auto C) {
            unroll<L::QY>([&](auto B) {
                unroll<L::QX>([&](auto A) {
                    constexpr int a = A, b = B, c = C;
                    v[c][b][a] = (float)(rho * Fx[a] * Fy[b] * Fz[c]);
                });
            });
        });
    }
    const uint32_t h = storage_hash<ST>(p.seed, i, y);
    unroll<L::QZ>([&](auto C) {
        unroll<L::QY>([&](auto B) {
            unroll<L::QX>([&](auto A) {
                constexpr int a = A, b = B, c = C;
                if constexpr (L::shifted) v[c][b][a] -= kShift3<LX, LY, LZ>.s[c][b][a];
                if constexpr (Elem<ST>::bytes == 2) v[c][b][a] = quantize<ST>(v[c][b][a], rnd_of<L::template q<a, b, c>()>(h));
            });
        });
    });
    const int row = z * p.ny + y;
    store3<LX, LY, LZ, ST, BCX>(p, make_rsrc(p.dst2, p.buf_bytes), x, row, v, h);
    float rho, jx, jy, jz;
    moments3<LX, LY, LZ, ST>(v, rho, jx, jy, jz);
    const float inv = 1.0f / rho;
    collide3<LX, LY, LZ, ST>(p, v, rho, jx, jy, jz, jx * inv, jy * inv, jz * inv, mix32(mix32(h)));
    store3<LX, LY, LZ, ST, BCX>(p, make_rsrc(p.dst, p.buf_bytes), x, row, v, mix32(h));
}

// FP64 sums (glbm_stats), as stats_kernel, with the z momentum in slot 11.
template <int LX, int LY, int LZ, int ST, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void stats3_kernel(KArgs p)
{
    using L = Lat3<LX, LY, LZ, ST>;
    double acc[kNumStats];
    for (int k = 0; k < kNumStats; ++k) acc[k] = 0.0;
    const rsrc_t rs = make_rsrc(p.src, p.buf_bytes);
    for (int i = blockIdx.x * kBlock + (int)threadIdx.x; i < p.nodes; i += gridDim.x * kBlock) {
        int x, y, z;
        node_xyz(p, i, x, y, z);
        const XAddr<LX, L::EB, BCX> xa(x, p.nx);
        const uint32_t base = xa.own(row_bytes<L::EB>(p, z * p.ny + y));
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0, e = 0.0;
        unroll<L::QZ>([&](auto C) {
            unroll<L::QY>([&](auto B) {
                unroll<L::QX>([&](auto A) {
                    constexpr int a = A, b = B, c = C, ca = Axis<LX>::c(a), cb = Axis<LY>::c(b), cc = Axis<LZ>::c(c);
                    const double f = ld<ST>(rs, base, (uint32_t)L::template q<a, b, c>() * p.plane_bytes);
                    r += f;
                    jx += ca * f;
                    jy += cb * f;
                    jz += cc * f;
                    e += (ca * ca + cb * cb + cc * cc) * f;
                });
            });
        });
        if constexpr (L::shifted) {
            r += (double)kShift3<LX, LY, LZ>.sum;
            e += (double)kShift3<LX, LY, LZ>.sxx + (double)kShift3<LX, LY, LZ>.syy + (double)kShift3<LX, LY, LZ>.szz;
        }
        const double jx_pre = jx - p.g;
        const double ux = jx_pre / r, uy = jy / r, uz = jz / r;
        acc[0] += r;
        acc[1] += jx_pre;
        acc[2] += jy;
        acc[3] += e;
        acc[4] += ux * ux;
        acc[11] += jz;
        if (p.prev) {
            const rsrc_t rp = make_rsrc(p.prev, p.buf_bytes);
            double r0 = 0.0, j0 = 0.0;
            unroll<L::QZ>([&](auto C) {
                unroll<L::QY>([&](auto B) {
                    unroll<L::QX>([&](auto A) {
                        constexpr int a = A, b = B, c = C;
                        const double f = ld<ST>(rp, base, (uint32_t)L::template q<a, b, c>() * p.plane_bytes);
                        r0 += f;
                        j0 += Axis<LX>::c(a) * f;
                    });
                });
            });
            if constexpr (L::shifted) r0 += (double)kShift3<LX, LY, LZ>.sum;
            const double d = ux - (j0 - p.g) / r0;
            acc[5] += d * d;
        }
        if (!finite_node(r, jx, jy, jz, e))
            acc[12] += 1.0;
        else if (ux * ux > Axis<LX>::u2max || uy * uy > Axis<LY>::u2max || uz * uz > Axis<LZ>::u2max)
            acc[10] += 1.0;
        if constexpr (BCY == BCY_WALL) {
            if (y == 0) {
                float m;
                const float A = wall_absorbed3<LX, LY, LZ, ST, BCX, true>(p, rs, xa, z, &m);
                acc[6] += A;
                acc[7] += (double)m - (double)A * p.uw[0];
            }
            if (y == p.ny - 1) {
                float m;
                const float A = wall_absorbed3<LX, LY, LZ, ST, BCX, false>(p, rs, xa, z, &m);
                acc[8] += A;
                acc[9] += (double)m - (double)A * p.uw[1];
            }
        }
    }
    write_partials(acc, p.partials);
}

}  // namespace glbm
