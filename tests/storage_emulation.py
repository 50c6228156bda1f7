"""CPU emulation of the population storages of the GPU path, to measure what
each rounding scheme costs against the FP64 oracle (test infrastructure).

A plain numpy stepper of the symmetric two-dimensional channel (G-D2Q((2N+1)^2),
periodic x, diffuse walls across y, linear force; the same readings as the
oracle: collide, wall densities from the absorbed populations, pull
streaming) whose post-collision state passes through a storage model after
every step.  With no rounding it reproduces the oracle to ~1e-14, so every
difference it shows comes from the storage.  It shares no code with the HIP
library or the oracle.

Storage models (``scheme``):
  f64              no rounding
  f32dev           FP32 deviation f - W, round to nearest (the update f + d,
                   rounded once)
  f32dev_dither    the same with the increment dithered by one unit in the
                   last place of the stored value (unbiased rounding; the
                   library's FP32 deviation storage)
  rest_sr/_rne     BF16 deviation from the rest state W, stochastic or nearest
                   rounding (the library's BF16 storages)
  lin_sr/_rne      BF16 deviation from the node's own first-order equilibrium
                   W (rho + c.j / theta) with rho, j kept in FP32 per node
  lin_*_cons       the same, the rounding defects of mass and momentum folded
                   back into the FP32 rho and j (conservative)
  eq_*_cons        BF16 deviation from the full local equilibrium, conservative
"""
from __future__ import annotations

import numpy as np


def axis_equilibrium(N: int, u):
    """Per-axis equilibrium at rho = 1: N-fold convolution of the D1Q3 step
    probabilities at u / N (entries n = -N..N along axis 0)."""
    v = np.asarray(u, dtype=np.float64) / N
    pp = 1 / 6 + 0.5 * v + 0.5 * v * v
    pm = 1 / 6 - 0.5 * v + 0.5 * v * v
    p0 = 2 / 3 - v * v
    F = [np.ones_like(v)]
    for _ in range(N):
        nxt = [np.zeros_like(v) for _ in range(len(F) + 2)]
        for i, x in enumerate(F):
            nxt[i] += pm * x
            nxt[i + 1] += p0 * x
            nxt[i + 2] += pp * x
        F = nxt
    return np.array(F)


def bf16_nearest(x):
    b = np.asarray(x, np.float32).view(np.uint32)
    lsb = (b >> 16) & 1
    return ((b + np.uint32(0x7FFF) + lsb) & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)


def bf16_stochastic(x, rng):
    b = np.asarray(x, np.float32).view(np.uint32)
    r = rng.integers(0, 1 << 16, size=b.shape, dtype=np.uint32)
    return ((b + r) & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


class Channel:
    """Symmetric level-N channel, nx x ny nodes, populations [b][a][y][x]."""

    def __init__(self, N, nx, ny, tau, wall_u=(0.0, 0.0), g=0.0, scheme="f64", seed=1):
        self.N, self.nx, self.ny = N, nx, ny
        self.Q1 = 2 * N + 1
        self.c = np.arange(-N, N + 1)
        self.W = axis_equilibrium(N, np.zeros(1))[:, 0]
        self.theta = N / 3.0
        self.omega = 1.0 / (tau + 0.5)
        self.g = g
        self.scheme = scheme
        self.rng = np.random.default_rng(seed)
        self.Jp = sum(n * self.W[N + n] for n in range(1, N + 1))  # half flux
        self.E = [axis_equilibrium(N, np.array([U]))[:, 0] for U in wall_u]
        self.W2 = np.outer(self.W, self.W)
        self.t = 0
        ones, zeros = np.ones((ny, nx)), np.zeros((ny, nx))
        self.fpre = self.feq(ones, zeros, zeros)
        self._store(self._collide(self.fpre))

    def feq(self, rho, ux, uy):
        return rho[None, None] * axis_equilibrium(self.N, uy)[:, None] * axis_equilibrium(self.N, ux)[None, :]

    def _moments(self, f):
        rho = f.sum(axis=(0, 1))
        return rho, np.einsum("bayx,a->yx", f, self.c), np.einsum("bayx,b->yx", f, self.c)

    def _collide(self, f):
        rho, jx, jy = self._moments(f)
        force = (self.W2 * self.c[None, :] * self.g / self.theta)[:, :, None, None]
        return f + self.omega * (self.feq(rho, jx / rho, jy / rho) - f) + force

    def _reference(self, rho, jx, jy):
        if self.scheme.startswith("eq"):
            return self.feq(rho, jx / rho, jy / rho)
        c = self.c
        return self.W2[:, :, None, None] * (rho[None, None] + (c[None, :, None, None] * jx[None, None]
                                                             + c[:, None, None, None] * jy[None, None]) / self.theta)

    def _round16(self, x):
        return bf16_stochastic(x, self.rng) if "_sr" in self.scheme else bf16_nearest(x)

    def _store(self, fs):
        s, W2 = self.scheme, np.broadcast_to(self.W2[:, :, None, None], fs.shape)
        if s == "f64":
            self.F = fs
        elif s == "f32dev":
            self.F = W2 + f32(fs - W2)
        elif s == "f32dev_dither":
            prev = f32(self.fpre - W2)
            inc = (fs - W2) - prev
            ulp = np.ldexp(1.0, np.frexp(prev.astype(np.float32))[1] - 24)
            d = (self.rng.random(size=fs.shape) - 0.5) * ulp
            self.F = W2 + f32(prev + f32(inc + d))
        elif s.startswith("rest"):
            self.F = W2 + self._round16(fs - W2)
        elif s.startswith("lin") or s.startswith("eq"):
            rho, jx, jy = (f32(v) for v in self._moments(fs))
            dev = f32(fs - self._reference(rho, jx, jy))
            q = self._round16(dev)
            if s.endswith("_cons"):
                d = q - dev
                rho = f32(rho - d.sum(axis=(0, 1)))
                jx = f32(jx - np.einsum("bayx,a->yx", d, self.c))
                jy = f32(jy - np.einsum("bayx,b->yx", d, self.c))
            self.F = self._reference(rho, jx, jy) + q
        else:
            raise ValueError(s)

    def _pull(self):
        F, N, nx, ny, c = self.F, self.N, self.nx, self.ny, self.c
        f = np.empty_like(F)
        rw = []
        for side in (0, 1):  # absorbed mass per column -> wall density
            A = np.zeros(nx)
            for b in range(self.Q1):
                if (side == 0 and c[b] < 0) or (side == 1 and c[b] > 0):
                    for r in range(abs(c[b])):
                        row = r if side == 0 else ny - 1 - r
                        for a in range(self.Q1):
                            A += np.roll(F[b, a, row], c[a])
            rw.append(A / self.Jp)
        for b in range(self.Q1):
            cb = c[b]
            for a in range(self.Q1):
                src = np.roll(F[b, a], c[a], axis=1)
                if cb > 0:
                    f[b, a, cb:] = src[:ny - cb]
                    f[b, a, :cb] = (rw[0] * self.E[0][a] * self.W[b])[None, :]
                elif cb < 0:
                    f[b, a, :ny + cb] = src[-cb:]
                    f[b, a, ny + cb:] = (rw[1] * self.E[1][a] * self.W[b])[None, :]
                else:
                    f[b, a] = src
        return f

    def step(self, n: int = 1):
        for _ in range(n):
            self.fpre = self._pull()
            self._store(self._collide(self.fpre))
            self.t += 1

    def moments(self) -> dict:
        f = self.fpre
        rho, jx, jy = self._moments(f)
        ux, uy = jx / rho, jy / rho
        c2 = self.c * self.c
        e2 = np.einsum("bayx,a->yx", f, c2) + np.einsum("bayx,b->yx", f, c2)
        pxy = np.einsum("bayx,a,b->yx", f, self.c, self.c) - rho * ux * uy
        return {"rho": rho, "ux": ux, "uy": uy, "T": (e2 / rho - ux * ux - uy * uy) / 2, "pxy": pxy}
