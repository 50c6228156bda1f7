"""Studies built on the library: the experiments of section 5 that need no
external data, run on the GPU through batches of lattices.

* ``sod_stability``: the Sod tube of section 5.1 (density 4 | 1, 800 nodes,
  theta0 = 1 in the paper's units, fixed equilibrium ends) over a grid of
  levels and viscosities, recording where the solution breaks down (a
  non-finite or non-positive density) and how strongly it oscillates.
* ``channel_observables``: steady Couette and force-driven Poiseuille
  channels over levels and Knudsen numbers (sections 5.3-5.4): slip
  velocity, normalised flow rate and the volumetric flow of section 5.4, for
  self-convergence in N and the Knudsen minimum of the even hierarchy at
  N >= 10 (the paper's benchmark curves are not available).

Units: the paper fixes theta0 = 1 and the lattice step c(N) per level; the
library works on each axis in its own lattice units (unit spacing, theta =
N/3 or (4N+3)/3).  The relaxation time tau is the same number in both (nu =
theta tau in either), so a viscosity nu of the paper is tau = nu here.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import glbm


def axis_theta(level: int, even: bool = False) -> float:
    return (4 * level + 3) / 3.0 if even else level / 3.0


# ------------------------------------------------------------------- Sod
@dataclasses.dataclass
class SodOutcome:
    level: int
    even: bool
    nu: float
    steps: int                 # steps run (the horizon, or up to the breakdown)
    broke_at: int | None       # first check (step) with a non-finite or non-positive density
    overshoot: float           # max rho - 4 at the end (nan after a breakdown)
    total_variation: float     # sum |rho(x+1) - rho(x)| at the end (oscillation measure)


def sod_horizon(level: int, even: bool = False, nodes: int = 800) -> int:
    """Steps for sound to cross a quarter of the tube (the same physical time
    for every level: the shock stays inside)."""
    return int(round(0.25 * nodes / math.sqrt(axis_theta(level, even))))


def sod_stability(levels=range(1, 8), nus=(0.1, 0.03, 0.02, 0.01, 0.005, 0.002, 0.001, 0.0005), even=False,
                  nodes: int = 800, storage: str = "f32_shifted", checks: int = 10):
    """One batch per level (all viscosities), stepped to the level's horizon
    in `checks` chunks; after each chunk the densities are checked."""
    import torch

    rho0 = np.where((np.arange(nodes) + 0.5) / nodes <= 0.5, 4.0, 1.0).astype(np.float32)
    out = []
    for lv in levels:
        T = sod_horizon(lv, even, nodes)
        chunk = max(1, T // checks)
        solvers = []
        for nu in nus:
            cfg = glbm.make_config(1, lv, 0, nodes, 1, tau=nu, bc_x="eq_ends", end_rho=(4.0, 1.0), storage=storage,
                                   even_x=even)
            s = glbm.Solver(cfg)
            s.init_fields(rho0, np.zeros_like(rho0))
            solvers.append(s)
        broke = [None] * len(nus)
        done = 0
        with glbm.Batch(solvers, resident_nodes=nodes) as b:
            for _ in range(checks):
                b.step(chunk)
                done += chunk
                for k, s in enumerate(solvers):
                    if broke[k] is None:
                        r = s.moments(("rho",))["rho"]
                        if not bool(torch.isfinite(r).all()) or float(r.min()) <= 0.0:
                            broke[k] = done
        for k, (nu, s) in enumerate(zip(nus, solvers)):
            r = s.moments(("rho",))["rho"][0].double().cpu().numpy()
            ok = broke[k] is None
            out.append(SodOutcome(lv, even, nu, done, broke[k], float(r.max() - 4.0) if ok else float("nan"),
                                  float(np.abs(np.diff(r)).sum()) if ok else float("nan")))
            s.close()
    return out


# --------------------------------------------------------------- channels
@dataclasses.dataclass
class ChannelOutcome:
    kind: str                  # couette | poiseuille
    lattice: str               # odd | mixed_even (D1Q3 x G-D1Q(2N+2))
    level: int
    kn: float
    steps: int
    residual: float            # steady-state residual at the end
    slip: float                # see channel_observables
    flow: float                # Couette: normalised wall shear stress; Poiseuille: normalised flow rate
    volumetric: float = float("nan")  # Poiseuille: the volumetric flow of section 5.4 (see channel_observables)


def channel_observables(kind: str, levels, kns, lattice: str = "mixed_even", ny: int = 64, steps: int = 20000,
                        storage: str = "f32_shifted", speed_cs: float = 0.01, resident: bool = True):
    """Steady channels of section 5.3 (Couette) or 5.4 (Poiseuille), one
    batch over all (level, Kn), nx = 4 (x-uniform flows, members resident),
    run `steps` steps from rest.  U = speed_cs times the sound speed of the
    wall-normal axis; H = ny (walls half way between nodes); nu = theta tau.

    Couette (walls at -U, +U):
      slip = (u(y_0) + U) / (2U) - 1/(2 ny): the fluid's speed at the first
        node relative to the wall, beyond the no-slip linear profile (0 in the
        continuum limit, 1/2 - 1/(2 ny) in the free-molecular one);
      flow = wall shear stress (x momentum taken up by the bottom wall per
        column and step) over its continuum value 2 U nu / H.
    Poiseuille (walls at rest, g = 8 nu U / H^2):
      slip = u(y_0) / u(y_centre);
      flow = sum_y u(y) / (2 U H / 3), the flow rate over the no-slip
        continuum value;
      volumetric = delta / (4 U H) sum_y u(y), the volumetric flow of section
        5.4 with U the no-slip centre-line speed g H^2 / (8 nu) and the
        rarefaction parameter delta = sqrt(pi) / (2 Kn) (the paper does not
        restate delta; this is the usual definition of the tabulated data it
        compares with)."""
    import torch

    confs, meta = [], []
    for lv in levels:
        for kn in kns:
            if lattice == "odd":
                lx, ly, ex, ey = lv, lv, False, False
            else:
                lx, ly, ex, ey = 1, lv, False, True
            th_y = axis_theta(ly, ey)
            U = speed_cs * math.sqrt(th_y)
            nu = th_y * kn * ny / math.sqrt(2 * th_y)
            if kind == "couette":
                cfg = glbm.make_config(2, lx, ly, 4, ny, kn=kn, bc_y="wall", wall_u=(-U, U), storage=storage,
                                       even_x=ex, even_y=ey)
            else:
                cfg = glbm.make_config(2, lx, ly, 4, ny, kn=kn, bc_y="wall", g=8 * nu * U / (ny * ny),
                                       storage=storage, even_x=ex, even_y=ey)
            confs.append(cfg)
            meta.append((lv, kn, U, nu))
    solvers = [glbm.Solver(c) for c in confs]
    for s in solvers:
        s.init_fields()
    torch.cuda.synchronize()
    with glbm.Batch(solvers, resident_nodes=4 * ny if resident else 0) as b:
        b.step(steps)
    out = []
    for s, (lv, kn, U, nu) in zip(solvers, meta):
        ux = s.moments(("ux",))["ux"][:, 0].double().cpu().numpy()
        st = s.stats()
        vol = float("nan")
        if kind == "couette":
            slip = (ux[0] + U) / (2 * U) - 0.5 / ny
            flow = (st["wall_momentum_bottom"] / 4) / (2 * U * nu / ny)
        else:
            slip = ux[0] / ux[ny // 2]
            flow = ux.sum() / (2.0 * U * ny / 3.0)
            vol = math.sqrt(math.pi) / (2.0 * kn) * ux.sum() / (4.0 * U * ny)
        out.append(ChannelOutcome(kind, lattice, lv, kn, steps, st["residual"], float(slip), float(flow), vol))
        s.close()
    return out
