"""ctypes binding of the FP64 oracle (``glbm_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Arrays use the
oracle's layout: populations ``[q][y][x]`` with ``q = b*Qx + a`` and velocity
``(cx[a], cy[b])`` (``velocities()``): ``a - N`` on a G-D1Q(2N+1) axis, the odd
integers ``2a - (2N+1)`` on a G-D1Q(2N+2) axis (grid of half the lattice
step); node fields ``[y][x]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

BC_PERIODIC = 0
BC_WALL = 1
BC_EQ_ENDS = 2
AXIS_ODD = 0
AXIS_EVEN = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "glbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math) into liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB):
            build_oracle(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.orc_equilibrium_1d.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        lib.orc_equilibrium_1d.restype = None
        lib.orc_step_probabilities.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        lib.orc_step_probabilities.restype = None
        lib.orc_tau_from_kn.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.orc_tau_from_kn.restype = ctypes.c_double
        lib.orc_axis_equilibrium.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp]
        lib.orc_axis_equilibrium.restype = None
        lib.orc_create.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_double,
        ]
        lib.orc_create.restype = ctypes.c_void_p
        lib.orc_create3.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_double,
        ]
        lib.orc_create3.restype = ctypes.c_void_p
        lib.orc_axis_velocities_z.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
        lib.orc_axis_velocities_z.restype = ctypes.c_int
        lib.orc_init_fields3.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        lib.orc_moments3.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.orc_destroy.argtypes = [ctypes.c_void_p]
        lib.orc_tau.argtypes = [ctypes.c_void_p]
        lib.orc_tau.restype = ctypes.c_double
        lib.orc_omega.argtypes = [ctypes.c_void_p]
        lib.orc_omega.restype = ctypes.c_double
        lib.orc_time.argtypes = [ctypes.c_void_p]
        lib.orc_time.restype = ctypes.c_int64
        lib.orc_nvel.argtypes = [ctypes.c_void_p]
        lib.orc_nvel.restype = ctypes.c_int
        lib.orc_tables.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        lib.orc_axis_velocities.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        lib.orc_axis_velocities.restype = ctypes.c_int
        lib.orc_init_fields.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        lib.orc_init_populations.argtypes = [ctypes.c_void_p, _dp]
        lib.orc_get_populations.argtypes = [ctypes.c_void_p, _dp]
        lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        lib.orc_moments.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp]
        lib.orc_stats.argtypes = [ctypes.c_void_p, _dp]
        _lib = lib
        return lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def equilibrium_1d(N: int, u: float, c: float = 1.0, theta0: float | None = None) -> np.ndarray:
    """Closed-form equilibrium (Eq. maineq03) at rho = 1 for n = -N..N.

    ``theta0`` defaults to the calibration N c^2 / 3 of Eq. maineq05."""
    lib = _load()
    if theta0 is None:
        theta0 = N * c * c / 3.0
    out = np.zeros(2 * N + 1)
    lib.orc_equilibrium_1d(int(N), float(c), float(theta0), float(u), _ptr(out))
    return out


def step_probabilities(N: int, u: float, c: float = 1.0, theta0: float | None = None) -> np.ndarray:
    """(P-, P0, P+) of Eq. maineq04."""
    lib = _load()
    if theta0 is None:
        theta0 = N * c * c / 3.0
    out = np.zeros(3)
    lib.orc_step_probabilities(int(N), float(c), float(theta0), float(u), _ptr(out))
    return out


def rest_weights(N: int, even: bool = False) -> np.ndarray:
    """Equilibrium at rho = 1, u = 0 (the weights W used by the force term)."""
    return axis_equilibrium(N, 0.0, even)


def axis_equilibrium(N: int, u: float, even: bool = False) -> np.ndarray:
    """Equilibrium at rho = 1 of an axis in lattice units (unit grid spacing):
    G-D1Q(2N+1) at velocities -N..N, or G-D1Q(2N+2) at the odd velocities
    -(2N+1)..2N+1 (Eqs. maineq01_noball-maineq04_noball)."""
    lib = _load()
    out = np.zeros(2 * N + 2 if even else 2 * N + 1)
    lib.orc_axis_equilibrium(AXIS_EVEN if even else AXIS_ODD, int(N), float(u), _ptr(out))
    return out


def axis_velocities(N: int, even: bool = False) -> np.ndarray:
    return np.arange(-(2 * N + 1), 2 * N + 2, 2) if even else np.arange(-N, N + 1)


def tau_from_kn(kn: float, H: float, theta: float) -> float:
    return _load().orc_tau_from_kn(float(kn), float(H), float(theta))


class OracleSolver:
    """One FP64 solver instance (see ``glbm_oracle.c`` for the step order)."""

    STAT_NAMES = (
        "mass", "momentum_x", "momentum_y", "energy_post", "residual",
        "wall_mass_bottom", "wall_mass_top", "wall_momentum_bottom", "wall_momentum_top",
        "nonpositive_nodes", "momentum_z", "nonfinite_nodes",
    )

    def __init__(self, dims, level_x, level_y=0, nx=1, ny=1, tau=0.0, kn=0.0,
                 bc_x=BC_PERIODIC, bc_y=BC_PERIODIC, wall_u=(0.0, 0.0), end_rho=(1.0, 1.0), g=0.0,
                 even_x=False, even_y=False, level_z=0, nz=1, even_z=False):
        """dims 1, 2 or 3; a third axis (level_z, nz, even_z) is periodic."""
        self._lib = _load()
        wu = np.asarray(wall_u, dtype=np.float64)
        er = np.asarray(end_rho, dtype=np.float64)
        h = self._lib.orc_create3(int(dims), int(level_x), int(level_y), int(level_z),
                                  AXIS_EVEN if even_x else AXIS_ODD, AXIS_EVEN if even_y else AXIS_ODD,
                                  AXIS_EVEN if even_z else AXIS_ODD, int(nx), int(ny), int(nz),
                                  float(tau), float(kn), int(bc_x), int(bc_y), _ptr(wu), _ptr(er), float(g))
        if not h:
            raise ValueError("oracle rejected the configuration")
        self._h = h
        self.dims = int(dims)
        self.level_x = int(level_x)
        self.level_y = int(level_y) if dims == 2 else 0
        self.level_z = int(level_z) if dims == 3 else 0
        self.nx = int(nx)
        self.ny = int(ny) if dims >= 2 else 1
        self.nz = int(nz) if dims == 3 else 1
        self.Q = self._lib.orc_nvel(h)
        cx = (ctypes.c_int * 64)()
        cy = (ctypes.c_int * 64)()
        cz = (ctypes.c_int * 64)()
        self.Qx = self._lib.orc_axis_velocities(h, cx, cy)
        self.Qz = self._lib.orc_axis_velocities_z(h, cz)
        self.Qy = self.Q // (self.Qx * self.Qz)
        self.cx = np.array(cx[:self.Qx])
        self.cy = np.array(cy[:self.Qy])
        self.cz = np.array(cz[:self.Qz])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    @property
    def tau(self):
        return self._lib.orc_tau(self._h)

    @property
    def omega(self):
        return self._lib.orc_omega(self._h)

    @property
    def time(self):
        return self._lib.orc_time(self._h)

    @property
    def nodes(self):
        return self.nx * self.ny * self.nz

    def _shape(self):
        return (self.nz, self.ny, self.nx) if self.dims == 3 else (self.ny, self.nx)

    def velocities(self):
        return self.cx.copy(), self.cy.copy()

    def tables(self):
        Wx = np.zeros(self.Qx)
        Wy = np.zeros(self.Qy)
        jp = np.zeros(1)
        self._lib.orc_tables(self._h, _ptr(Wx), _ptr(Wy), _ptr(jp))
        return Wx, Wy, float(jp[0])

    def init_fields(self, rho=None, ux=None, uy=None, uz=None):
        n = self.nodes
        r, a, b, c = _f64(rho, n), _f64(ux, n), _f64(uy, n), _f64(uz, n)
        self._lib.orc_init_fields3(self._h, _ptr(r), _ptr(a), _ptr(b), _ptr(c))

    def init_populations(self, f0):
        f0 = _f64(f0, self.Q * self.nodes)
        self._lib.orc_init_populations(self._h, _ptr(f0))

    def populations(self) -> np.ndarray:
        out = np.zeros(self.Q * self.nodes)
        self._lib.orc_get_populations(self._h, _ptr(out))
        return out.reshape((self.Q,) + self._shape())

    def step(self, n: int = 1):
        self._lib.orc_step(self._h, int(n))

    def moments(self) -> dict:
        """rho, ux, uy, T, pxy (and uz in three dimensions), shaped like the lattice."""
        n = self.nodes
        keys = ("rho", "ux", "uy", "uz", "T", "pxy")
        out = {k: np.zeros(n) for k in keys}
        self._lib.orc_moments3(self._h, *[_ptr(out[k]) for k in keys])
        if self.dims < 3:
            del out["uz"]
        return {k: v.reshape(self._shape()) for k, v in out.items()}

    def stats(self) -> dict:
        out = np.zeros(len(self.STAT_NAMES))
        self._lib.orc_stats(self._h, _ptr(out))
        return dict(zip(self.STAT_NAMES, out.tolist()))
