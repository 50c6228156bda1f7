"""Literal push-form stepper for tiny lattices (test-only).

An independent second reading of one time step, written without numpy and
without the oracle: dictionaries keyed by (x, y, c_x, c_y), the equilibrium
obtained by enumerating the 3^N outcomes of the dice problem of section 2,
collision at every node (Eq. maineq01, linear force of section 5.4), then
each post-collision population *pushed* to x + c.  Populations pushed
through a diffuse wall are absorbed per destination column and re-emitted as
the unit-density equilibrium at the wall velocity scaled so that the column
keeps its mass; populations pushed out of a fixed-equilibrium end are lost
and the end supplies equilibrium populations at rest.

An axis is a G-D1Q(2N+1) axis (velocities -N..N) or, with ``even``, a
G-D1Q(2N+2) axis on the grid of half its lattice step: velocities the odd
integers up to 2N+1, its equilibrium the law of the N-step sum on the
doubled lattice (steps -2, 0, 2) plus an independent fair step of -1 or +1
(the neighbour average of section 2, read as a random walk).
"""
from __future__ import annotations

import itertools
from collections import defaultdict

PERIODIC, WALL, EQ_ENDS = 0, 1, 2


def dice_law(N: int, u: float) -> dict:
    """Sum of N steps in {-1, 0, 1} with mean u/N and variance (N/3)/N each."""
    if N == 0:
        return {0: 1.0}
    mean = u / N
    second = (N / 3.0) / N + mean * mean
    p = {1: 0.5 * (second + mean), -1: 0.5 * (second - mean)}
    p[0] = 1.0 - p[1] - p[-1]
    law = defaultdict(float)
    for steps in itertools.product((-1, 0, 1), repeat=N):
        prob = 1.0
        for s in steps:
            prob *= p[s]
        law[sum(steps)] += prob
    return dict(law)


def even_law(N: int, u: float) -> dict:
    """Sum of N steps in {-2, 0, 2} (mean u/N, the doubled lattice of
    temperature 4N/3) plus a fair step in {-1, +1}."""
    half = dice_law(N, u / 2.0)
    law = defaultdict(float)
    for k, p in half.items():
        law[2 * k + 1] += 0.5 * p
        law[2 * k - 1] += 0.5 * p
    return dict(law)


def axis_law(N: int, even: bool, u: float) -> dict:
    return even_law(N, u) if even else dice_law(N, u)


def axis_velocities(N: int, even: bool):
    return list(range(-(2 * N + 1), 2 * N + 2, 2)) if even else list(range(-N, N + 1))


def run(dims, Lx, Ly, nx, ny, omega, g, bc_x, bc_y, wall_u, end_rho, f0, steps, even_x=False, even_y=False):
    """Advance ``f0`` (a dict {(x, y, cx, cy): value}) by ``steps`` steps."""
    if dims == 1:
        Ly, ny, bc_y, even_y = 0, 1, PERIODIC, False
    vel = [(cx, cy) for cy in axis_velocities(Ly, even_y) for cx in axis_velocities(Lx, even_x)]
    Wx, Wy = axis_law(Lx, even_x, 0.0), axis_law(Ly, even_y, 0.0)
    thx = sum(Wx[c] * c * c for c in Wx)  # axis temperature: second moment at rest
    jplus = sum(cy * Wy[cy] for cy in Wy if cy > 0)
    Fbot, Ftop = axis_law(Lx, even_x, wall_u[0]), axis_law(Lx, even_x, wall_u[1])
    f = dict(f0)
    for _ in range(steps):
        post = {}
        for x in range(nx):
            for y in range(ny):
                rho = sum(f[(x, y, cx, cy)] for cx, cy in vel)
                ux = sum(f[(x, y, cx, cy)] * cx for cx, cy in vel) / rho
                uy = sum(f[(x, y, cx, cy)] * cy for cx, cy in vel) / rho
                ex, ey = axis_law(Lx, even_x, ux), axis_law(Ly, even_y, uy)
                for cx, cy in vel:
                    v = f[(x, y, cx, cy)]
                    feq = rho * ex[cx] * ey[cy]
                    force = Wx[cx] * Wy[cy] * cx * g / thx
                    post[(x, y, cx, cy)] = v + omega * (feq - v) + force
        new = {}
        absorbed = {"bot": defaultdict(float), "top": defaultdict(float)}
        for (x, y, cx, cy), v in post.items():
            xd, yd = x + cx, y + cy
            if bc_y == WALL and yd < 0:
                absorbed["bot"][xd % nx] += v
                continue
            if bc_y == WALL and yd >= ny:
                absorbed["top"][xd % nx] += v
                continue
            yd %= ny
            if bc_x == EQ_ENDS and not (0 <= xd < nx):
                continue
            new[(xd % nx, yd, cx, cy)] = v
        if bc_y == WALL:
            for x in range(nx):
                for cx, cy in vel:
                    if cy > 0:
                        for y in range(cy):
                            new[(x, y, cx, cy)] = absorbed["bot"][x] / jplus * Fbot[cx] * Wy[cy]
                    elif cy < 0:
                        for y in range(ny + cy, ny):
                            new[(x, y, cx, cy)] = absorbed["top"][x] / jplus * Ftop[cx] * Wy[cy]
        if bc_x == EQ_ENDS:
            for y in range(ny):
                for cx, cy in vel:
                    for x in range(0, min(cx, nx)):
                        new[(x, y, cx, cy)] = end_rho[0] * Wx[cx] * Wy[cy]
                    for x in range(max(nx + cx, 0), nx):
                        new[(x, y, cx, cy)] = end_rho[1] * Wx[cx] * Wy[cy]
        assert len(new) == len(vel) * nx * ny
        f = new
    return f


def to_dict(arr, Lx, Ly, even_x=False, even_y=False):
    """[q][y][x] array (q = b*Qx + a, velocities in increasing order per axis)
    -> dict keyed by (x, y, cx, cy)."""
    vx, vy = axis_velocities(Lx, even_x), axis_velocities(Ly, even_y)
    Q, ny, nx = arr.shape
    out = {}
    for q in range(Q):
        b, a = divmod(q, len(vx))
        for y in range(ny):
            for x in range(nx):
                out[(x, y, vx[a], vy[b])] = float(arr[q, y, x])
    return out


def from_dict(d, Lx, Ly, nx, ny, even_x=False, even_y=False):
    import numpy as np

    vx, vy = axis_velocities(Lx, even_x), axis_velocities(Ly, even_y)
    ix = {c: i for i, c in enumerate(vx)}
    iy = {c: i for i, c in enumerate(vy)}
    arr = np.zeros((len(vx) * len(vy), ny, nx))
    for (x, y, cx, cy), v in d.items():
        arr[iy[cy] * len(vx) + ix[cx], y, x] = v
    return arr


def run3(Lx, Ly, Lz, nx, ny, nz, omega, g, bc_y, wall_u, f0, steps, even=(False, False, False)):
    """Three dimensions (periodic x and z, y periodic or diffuse walls):
    ``f0`` is a dict {(x, y, z, cx, cy, cz): value}."""
    ex, ey, ez = even
    vel = [(cx, cy, cz) for cz in axis_velocities(Lz, ez) for cy in axis_velocities(Ly, ey)
           for cx in axis_velocities(Lx, ex)]
    Wx, Wy, Wz = axis_law(Lx, ex, 0.0), axis_law(Ly, ey, 0.0), axis_law(Lz, ez, 0.0)
    thx = sum(Wx[c] * c * c for c in Wx)
    jplus = sum(cy * Wy[cy] for cy in Wy if cy > 0)
    Fbot, Ftop = axis_law(Lx, ex, wall_u[0]), axis_law(Lx, ex, wall_u[1])
    nodes = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]
    f = dict(f0)
    for _ in range(steps):
        post = {}
        for x, y, z in nodes:
            vals = [(c, f[(x, y, z) + c]) for c in vel]
            rho = sum(v for _, v in vals)
            u = [sum(v * c[d] for c, v in vals) / rho for d in range(3)]
            ex_, ey_, ez_ = axis_law(Lx, ex, u[0]), axis_law(Ly, ey, u[1]), axis_law(Lz, ez, u[2])
            for c, v in vals:
                feq = rho * ex_[c[0]] * ey_[c[1]] * ez_[c[2]]
                force = Wx[c[0]] * Wy[c[1]] * Wz[c[2]] * c[0] * g / thx
                post[(x, y, z) + c] = v + omega * (feq - v) + force
        new = {}
        absorbed = {"bot": defaultdict(float), "top": defaultdict(float)}
        for (x, y, z, cx, cy, cz), v in post.items():
            xd, yd, zd = (x + cx) % nx, y + cy, (z + cz) % nz
            if bc_y == WALL and yd < 0:
                absorbed["bot"][(xd, zd)] += v
                continue
            if bc_y == WALL and yd >= ny:
                absorbed["top"][(xd, zd)] += v
                continue
            new[(xd, yd % ny, zd, cx, cy, cz)] = v
        if bc_y == WALL:
            for z in range(nz):
                for x in range(nx):
                    for cx, cy, cz in vel:
                        if cy > 0:
                            for y in range(cy):
                                new[(x, y, z, cx, cy, cz)] = absorbed["bot"][(x, z)] / jplus * Fbot[cx] * Wy[cy] * Wz[cz]
                        elif cy < 0:
                            for y in range(ny + cy, ny):
                                new[(x, y, z, cx, cy, cz)] = absorbed["top"][(x, z)] / jplus * Ftop[cx] * Wy[cy] * Wz[cz]
        assert len(new) == len(vel) * nx * ny * nz
        f = new
    return f


def to_dict3(arr, Lx, Ly, Lz, even=(False, False, False)):
    """[q][z][y][x] array, q = (c*Qy + b)*Qx + a -> dict keyed by (x, y, z, cx, cy, cz)."""
    vx, vy, vz = axis_velocities(Lx, even[0]), axis_velocities(Ly, even[1]), axis_velocities(Lz, even[2])
    Q, nz, ny, nx = arr.shape
    out = {}
    for q in range(Q):
        cb, a = divmod(q, len(vx))
        c, b = divmod(cb, len(vy))
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    out[(x, y, z, vx[a], vy[b], vz[c])] = float(arr[q, z, y, x])
    return out


def from_dict3(d, Lx, Ly, Lz, nx, ny, nz, even=(False, False, False)):
    import numpy as np

    vx, vy, vz = axis_velocities(Lx, even[0]), axis_velocities(Ly, even[1]), axis_velocities(Lz, even[2])
    ix = {c: i for i, c in enumerate(vx)}
    iy = {c: i for i, c in enumerate(vy)}
    iz = {c: i for i, c in enumerate(vz)}
    arr = np.zeros((len(vx) * len(vy) * len(vz), nz, ny, nx))
    for (x, y, z, cx, cy, cz), v in d.items():
        arr[(iz[cz] * len(vy) + iy[cy]) * len(vx) + ix[cx], z, y, x] = v
    return arr
