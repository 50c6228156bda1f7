"""Seeded synthetic workloads (sizes, parameters, initial fields).

This module only describes inputs: lattice sizes, boundary kinds, Knudsen
numbers, wall speeds, forces and seeded initial fields or populations.  It
holds none of the method's arithmetic, so that the HIP library and the FP64
oracle can both be fed from it without sharing any computation.

All random arrays are float32 values (returned as float64 copies where a
consumer wants FP64) so that the FP32 library and the FP64 oracle start from
bit-identical numbers.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Workload:
    name: str
    dims: int
    level_x: int            # hierarchy level N of the x axis (2N+1 velocities)
    level_y: int            # level of the y axis (0 in one dimension)
    nx: int
    ny: int
    kn: float = 0.0         # Knudsen number (used when tau <= 0)
    tau: float = 0.0        # relaxation time in lattice units (> 0 overrides kn)
    bc_x: str = "periodic"  # periodic | eq_ends
    bc_y: str = "periodic"  # periodic | wall
    wall_u: tuple = (0.0, 0.0)   # x velocity of the bottom / top wall (lattice units)
    end_rho: tuple = (1.0, 1.0)  # densities of the fixed equilibrium ends
    g: float = 0.0          # body force along x per node and step
    steps: int = 0
    storage: str = "f32"    # f32 | f32_shifted | bf16_shifted
    init: str = "rest"      # rest | sod | fields | populations
    even_x: bool = False    # G-D1Q(2N+2) velocity set on x (zero velocity removed)
    even_y: bool = False    # ... on y

    @property
    def nvel(self) -> int:
        qx = 2 * self.level_x + (2 if self.even_x else 1)
        qy = 1 if self.dims == 1 else 2 * self.level_y + (2 if self.even_y else 1)
        return qx * qy

    @property
    def nodes(self) -> int:
        return self.nx * self.ny


def sound_speed(level: int) -> float:
    """Lattice sound speed of a level-N axis with unit lattice spacing (sqrt(N/3))."""
    return math.sqrt(level / 3.0)


# -------------------------------------------------------------- recipes
def sod(nodes: int = 2000, level: int = 3, kn: float = 0.01, steps: int = 1000,
        rho_left: float = 1.0, rho_right: float = 0.125, storage: str = "f32") -> Workload:
    """1D shock tube: density step at the middle, fixed equilibrium ends.

    Default: D1Q7 (N = 3), 2000 nodes, densities 1 | 0.125, Kn = 0.01, 1000 steps."""
    return Workload("sod", 1, level, 0, nodes, 1, kn=kn, bc_x="eq_ends",
                    end_rho=(rho_left, rho_right), steps=steps, storage=storage, init="sod")


def couette(kn: float, ny: int = 256, nx: int = 4, level: int = 3, steps: int = 0,
            wall_speed_cs: float = 0.1, storage: str = "f32") -> Workload:
    """Plane Couette flow: walls at -U (bottom) and +U (top), U = 0.1 c_s, periodic x."""
    U = wall_speed_cs * sound_speed(level)
    return Workload("couette", 2, level, level, nx, ny, kn=kn, bc_y="wall",
                    wall_u=(-U, U), steps=steps, storage=storage)


def poiseuille(nx: int = 4096, ny: int = 1024, level: int = 5, kn: float = 0.1,
               g: float = 1e-5, steps: int = 20000, storage: str = "f32") -> Workload:
    """Force-driven channel between resting diffuse walls, periodic x.

    Default: D2Q(11x11) (N = 5 per axis), 4096 x 1024, g = 1e-5, Kn = 0.1."""
    return Workload("poiseuille", 2, level, level, nx, ny, kn=kn, bc_y="wall",
                    g=g, steps=steps, storage=storage)


# ------------------------------------------------------- seeded fields
def sod_density(nodes: int, rho_left: float, rho_right: float) -> np.ndarray:
    """Node i sits at (i + 1/2)/nodes on [0, 1]; left state for x < 1/2."""
    xc = (np.arange(nodes) + 0.5) / nodes
    return np.where(xc < 0.5, rho_left, rho_right).astype(np.float32)


def random_fields(seed: int, nx: int, ny: int, rho_amp: float = 0.05, u_amp: float = 0.05,
                  dims: int = 2):
    """Smooth-free random density/velocity fields (float32), rho near 1."""
    rng = np.random.default_rng(seed)
    rho = (1.0 + rho_amp * rng.uniform(-1, 1, size=(ny, nx))).astype(np.float32)
    ux = (u_amp * rng.uniform(-1, 1, size=(ny, nx))).astype(np.float32)
    uy = (u_amp * rng.uniform(-1, 1, size=(ny, nx))).astype(np.float32)
    if dims == 1:
        uy[:] = 0
    return rho, ux, uy


def wave_fields(nx: int, ny: int, rho_amp: float = 0.01, u_amp: float = 0.05, dims: int = 2):
    """Smooth periodic fields (float32): one sine period of density and shear
    across y, and of the y velocity along x."""
    y = (np.arange(ny) + 0.5) / ny
    x = (np.arange(nx) + 0.5) / nx
    Y, X = np.meshgrid(y, x, indexing="ij")
    rho = (1.0 + rho_amp * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)).astype(np.float32)
    ux = (u_amp * np.sin(2 * np.pi * Y)).astype(np.float32)
    uy = (0.5 * u_amp * np.cos(2 * np.pi * X)).astype(np.float32)
    if dims == 1:
        ux = (u_amp * np.sin(2 * np.pi * X)).astype(np.float32)
        uy[:] = 0
    return rho, ux, uy


def random_populations(seed: int, nvel: int, nx: int, ny: int, spread: float = 0.5) -> np.ndarray:
    """Positive random populations [q][y][x] (float32), each in (1 +- spread)/nvel."""
    rng = np.random.default_rng(seed)
    f = (1.0 + spread * rng.uniform(-1, 1, size=(nvel, ny, nx))) / nvel
    return f.astype(np.float32)


def batch_sweep(count: int = 512, seed: int = 190504597, steps: int = 2000):
    """Uneven channel instances: Couette or Poiseuille with equal odds, Ny ~ U{32..1024},
    Nx = 4, level ~ U{2..6} (k = level - 1 in 1..5), log10 Kn ~ U[-3, 1],
    speed ~ U[0.01, 0.1] c_s (the wall speed, or the target centre-line speed of
    a force-driven channel, g = 8 nu U / H^2 with nu = theta tau computed by the
    consumer)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = "couette" if rng.uniform() < 0.5 else "poiseuille"
        ny = int(rng.integers(32, 1025))
        level = int(rng.integers(2, 7))
        kn = float(10 ** rng.uniform(-3, 1))
        speed = float(rng.uniform(0.01, 0.1)) * sound_speed(level)
        out.append(dict(kind=kind, ny=ny, nx=4, level=level, kn=kn, speed=speed, steps=steps, index=i))
    return out


def sweep_workloads(count: int = 512, seed: int = 190504597, steps: int = 2000,
                    storage: str = "f32_shifted"):
    """The batched sweep as Workload objects (same draw as batch_sweep).

    Couette: walls at -/+ speed.  Poiseuille: walls at rest and the force
    that gives the drawn centre-line speed in the continuum limit,
    g = 8 nu U / H^2 with H = Ny, nu = theta tau, theta = N / 3 and the
    relaxation time that the Knudsen number sets, tau = Kn H / sqrt(2 theta)
    (an input recipe: the solvers derive tau from Kn themselves)."""
    out = []
    for d in batch_sweep(count, seed, steps):
        if d["kind"] == "couette":
            w = couette(d["kn"], ny=d["ny"], nx=d["nx"], level=d["level"], steps=steps, storage=storage)
            w.wall_u = (-d["speed"], d["speed"])
        else:
            theta = d["level"] / 3.0
            H = float(d["ny"])
            nu = theta * d["kn"] * H / math.sqrt(2.0 * theta)
            w = poiseuille(nx=d["nx"], ny=d["ny"], level=d["level"], kn=d["kn"],
                           g=8.0 * nu * d["speed"] / (H * H), steps=steps, storage=storage)
        w.name = "%s_%d" % (w.name, d["index"])
        out.append(w)
    return out


def log_uniform(rng, lo: float, hi: float) -> float:
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def served_requests(rate: float = 200.0, duration: float = 12.0, arrival_seed: int = 1905,
                    param_seed: int = 4597, sod_steps: int = 1000, channel_steps: int = 200,
                    storages=("f32_shifted", "bf16_shifted_sr")):
    """The served mix: Poisson arrivals at `rate` per second over `duration`
    seconds (arrival seed), each a Sod, Couette or Poiseuille solve with equal
    odds (parameter seed): level N ~ U{1..7} (k = N - 1 in 0..6), log10 Kn ~
    U[-3, 1], storage FP32 or BF16 deviations with equal odds; Sod over
    log-uniform 500..20000 nodes for `sod_steps` steps; channels with Ny and
    Nx log-uniform in [32, 2048] and [4, 2048], wall speed (Couette) or
    centre-line speed (Poiseuille) ~ U[0.01, 0.1] c_s, `channel_steps` steps.
    Every request draws all fields, so the parameter stream does not depend
    on the drawn kinds.  Returns [(arrival seconds, Workload)]."""
    ra = np.random.default_rng(arrival_seed)
    rp = np.random.default_rng(param_seed)
    out = []
    t = 0.0
    while True:
        t += float(ra.exponential(1.0 / rate))
        if t >= duration:
            break
        kind = ("sod", "couette", "poiseuille")[int(rp.integers(0, 3))]
        level = int(rp.integers(1, 8))
        kn = float(10 ** rp.uniform(-3, 1))
        storage = storages[int(rp.integers(0, len(storages)))]
        sod_nodes = int(round(log_uniform(rp, 500, 20000)))
        ny = int(round(log_uniform(rp, 32, 2048)))
        nx = int(round(log_uniform(rp, 4, 2048)))
        speed = float(rp.uniform(0.01, 0.1)) * sound_speed(level)
        if kind == "sod":
            w = sod(sod_nodes, level=level, kn=kn, steps=sod_steps, storage=storage)
        elif kind == "couette":
            w = couette(kn, ny=ny, nx=nx, level=level, steps=channel_steps, storage=storage)
            w.wall_u = (-speed, speed)
        else:
            theta = level / 3.0
            nu = theta * kn * ny / math.sqrt(2.0 * theta)
            w = poiseuille(nx=nx, ny=ny, level=level, kn=kn, g=8.0 * nu * speed / (ny * ny),
                           steps=channel_steps, storage=storage)
        w.name = "%s_%d" % (kind, len(out))
        out.append((t, w))
    return out


def maybe_f64(a: Optional[np.ndarray]):
    return None if a is None else np.asarray(a, dtype=np.float64)
