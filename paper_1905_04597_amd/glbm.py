"""ctypes binding of libglbm.so (the C-ABI declared in ``include/glbm.h``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  There is no
fallback: if the library or a GPU is missing, :func:`load` and
:class:`Solver` raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libglbm.so")

OK = 0
ERR_NONFINITE = -5
ERR_POSITIVITY = -6
# health of a state as glbm_stats reports it
HEALTH = {OK: "ok", ERR_NONFINITE: "nonfinite", ERR_POSITIVITY: "positivity"}
BC = {"periodic": 0, "wall": 1, "eq_ends": 2}
AXIS_ODD, AXIS_EVEN = 0, 1
STORAGE = {"f32": 0, "f32_shifted": 1, "bf16_shifted": 2, "bf16_shifted_sr": 3}
MAX_LEVEL = 13          # the even axis across the walls of the mixed lattices
MAX_LEVEL_ANY_AXIS = 7  # every other axis

# Exported entry points of include/glbm.h (kept in sync by tests/test_abi.py).
SYMBOLS = (
    "glbm_population_bytes", "glbm_create", "glbm_init_fields", "glbm_init_populations",
    "glbm_step", "glbm_moments", "glbm_get_populations", "glbm_stats", "glbm_info",
    "glbm_destroy", "glbm_last_error", "glbm_batch_create", "glbm_batch_step", "glbm_batch_destroy",
    "glbm_batch_update", "glbm_init_fields3", "glbm_moments3", "glbm_required_bytes",
    "glbm_stats_static", "glbm_bandwidth_probe",
)
ORDER = {"member": 0, "interleave": 1, "largest_first": 2}


class GlbmError(RuntimeError):
    pass


class Config(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int32),
        ("level_x", ctypes.c_int32),
        ("level_y", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("tau", ctypes.c_double),
        ("kn", ctypes.c_double),
        ("bc_x", ctypes.c_int32),
        ("bc_y", ctypes.c_int32),
        ("wall_u", ctypes.c_double * 2),
        ("end_rho", ctypes.c_double * 2),
        ("g", ctypes.c_double),
        ("kind_x", ctypes.c_int32),
        ("kind_y", ctypes.c_int32),
        ("nz", ctypes.c_int64),
        ("level_z", ctypes.c_int32),
        ("kind_z", ctypes.c_int32),
    ]


class BatchOptions(ctypes.Structure):
    _fields_ = [
        ("tile_nodes", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("graph_steps", ctypes.c_int32),
        ("resident_nodes", ctypes.c_int32),
        ("streams", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("time", ctypes.c_int64),
        ("mass", ctypes.c_double),
        ("momentum_x", ctypes.c_double),
        ("momentum_y", ctypes.c_double),
        ("energy_post", ctypes.c_double),
        ("residual", ctypes.c_double),
        ("wall_mass", ctypes.c_double * 2),
        ("wall_momentum", ctypes.c_double * 2),
        ("nonpositive_nodes", ctypes.c_double),
        ("momentum_z", ctypes.c_double),
        ("nonfinite_nodes", ctypes.c_double),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load libglbm.so (raises GlbmError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise GlbmError("libglbm.so not found at %s: run `python -m paper_1905_04597_amd.build`" % path)
    lib = ctypes.CDLL(path)
    vp, cp = ctypes.c_void_p, ctypes.POINTER(Config)
    lib.glbm_population_bytes.argtypes = [cp]
    lib.glbm_population_bytes.restype = ctypes.c_size_t
    lib.glbm_required_bytes.argtypes = [cp]
    lib.glbm_required_bytes.restype = ctypes.c_size_t
    lib.glbm_create.argtypes = [cp, vp, vp, vp, ctypes.POINTER(vp)]
    lib.glbm_create.restype = ctypes.c_int
    lib.glbm_init_fields.argtypes = [vp, vp, vp, vp]
    lib.glbm_init_populations.argtypes = [vp, vp]
    lib.glbm_step.argtypes = [vp, ctypes.c_int64]
    lib.glbm_moments.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.glbm_init_fields3.argtypes = [vp, vp, vp, vp, vp]
    lib.glbm_moments3.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.glbm_get_populations.argtypes = [vp, vp]
    lib.glbm_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.glbm_stats_static.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.glbm_bandwidth_probe.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_size_t, ctypes.c_int32, vp]
    lib.glbm_bandwidth_probe.restype = ctypes.c_int
    lib.glbm_info.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
    lib.glbm_destroy.argtypes = [vp]
    lib.glbm_last_error.argtypes = []
    lib.glbm_last_error.restype = ctypes.c_char_p
    lib.glbm_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(BatchOptions), vp,
                                      ctypes.POINTER(vp)]
    lib.glbm_batch_step.argtypes = [vp, ctypes.c_int64]
    lib.glbm_batch_update.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_int32]
    lib.glbm_batch_destroy.argtypes = [vp]
    for name in ("glbm_init_fields", "glbm_init_populations", "glbm_step", "glbm_moments",
                 "glbm_get_populations", "glbm_stats", "glbm_info", "glbm_destroy",
                 "glbm_batch_create", "glbm_batch_step", "glbm_batch_destroy", "glbm_batch_update",
                 "glbm_init_fields3", "glbm_moments3", "glbm_stats_static"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != OK:
        msg = load().glbm_last_error().decode(errors="replace")
        raise GlbmError("%s failed (%d): %s" % (what, rc, msg))


def make_config(dims, level_x, level_y=0, nx=1, ny=1, tau=0.0, kn=0.0, bc_x="periodic", bc_y="periodic",
                wall_u=(0.0, 0.0), end_rho=(1.0, 1.0), g=0.0, storage="f32", even_x=False, even_y=False,
                level_z=0, nz=1, even_z=False) -> Config:
    """even_x / even_y / even_z select the G-D1Q(2N+2) velocity set (zero
    velocity removed) for that axis instead of G-D1Q(2N+1); dims = 3 adds a
    periodic z axis (level_z, nz)."""
    c = Config()
    c.dims = int(dims)
    c.level_x = int(level_x)
    c.level_y = int(level_y)
    c.storage = STORAGE[storage]
    c.nx = int(nx)
    c.ny = int(ny)
    c.tau = float(tau)
    c.kn = float(kn)
    c.bc_x = BC[bc_x]
    c.bc_y = BC[bc_y]
    c.wall_u[0], c.wall_u[1] = float(wall_u[0]), float(wall_u[1])
    c.end_rho[0], c.end_rho[1] = float(end_rho[0]), float(end_rho[1])
    c.g = float(g)
    c.kind_x = AXIS_EVEN if even_x else AXIS_ODD
    c.kind_y = AXIS_EVEN if even_y else AXIS_ODD
    c.nz = int(nz)
    c.level_z = int(level_z)
    c.kind_z = AXIS_EVEN if even_z else AXIS_ODD
    return c


def config_from_workload(w) -> Config:
    return make_config(w.dims, w.level_x, w.level_y, w.nx, w.ny, w.tau, w.kn, w.bc_x, w.bc_y,
                       w.wall_u, w.end_rho, w.g, w.storage, getattr(w, "even_x", False), getattr(w, "even_y", False))


def population_bytes(cfg: Config) -> int:
    n = load().glbm_population_bytes(ctypes.byref(cfg))
    if n == 0:
        raise GlbmError("invalid configuration: " + load().glbm_last_error().decode(errors="replace"))
    return int(n)


def required_bytes(cfg: Config) -> int:
    """Device bytes of a solver: both population buffers and the statistics
    buffers (glbm_required_bytes)."""
    n = load().glbm_required_bytes(ctypes.byref(cfg))
    if n == 0:
        raise GlbmError("invalid configuration: " + load().glbm_last_error().decode(errors="replace"))
    return int(n)


class Solver:
    """One lattice on one GPU.

    Buffers are two PyTorch uint8 tensors owned by this object; all work is
    enqueued on ``stream`` (default: the current torch stream of ``device``).
    """

    def __init__(self, cfg: Config, device=None, stream=None, buffers=None):
        import torch

        if not torch.cuda.is_available():
            raise GlbmError("no GPU available: the glbm library has no CPU path")
        self._torch = torch
        self.lib = load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.cfg = cfg
        self.nbytes = population_bytes(cfg)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            if buffers is None:
                buffers = [torch.empty(self.nbytes, dtype=torch.uint8, device=self.device) for _ in range(2)]
            self.buffers = buffers
            h = ctypes.c_void_p()
            _check(self.lib.glbm_create(ctypes.byref(cfg), buffers[0].data_ptr(), buffers[1].data_ptr(),
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "glbm_create")
        self._h = h
        self.dims = cfg.dims
        self.nx = int(cfg.nx)
        self.ny = int(cfg.ny) if cfg.dims >= 2 else 1
        self.nz = int(cfg.nz) if cfg.dims == 3 else 1
        self.level_x = int(cfg.level_x)
        self.level_y = int(cfg.level_y) if cfg.dims >= 2 else 0
        self.level_z = int(cfg.level_z) if cfg.dims == 3 else 0
        qx = 2 * self.level_x + (2 if cfg.kind_x == AXIS_EVEN else 1)
        qy = 1 if cfg.dims == 1 else 2 * self.level_y + (2 if cfg.kind_y == AXIS_EVEN else 1)
        qz = 1 if cfg.dims < 3 else 2 * self.level_z + (2 if cfg.kind_z == AXIS_EVEN else 1)
        self.Q = qx * qy * qz
        self.shape = (self.nz, self.ny, self.nx) if cfg.dims == 3 else (self.ny, self.nx)
        self._keep = []

    # ------------------------------------------------------------- helpers
    def _dev(self, a, shape):
        torch = self._torch
        if a is None:
            return None
        t = torch.as_tensor(a, dtype=torch.float32).to(self.device).contiguous()
        if t.numel() != int(torch.tensor(shape).prod()):
            raise GlbmError("expected %s values, got %d" % (shape, t.numel()))
        return t

    @staticmethod
    def _ptr(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    # ---------------------------------------------------------------- API
    def init_fields(self, rho=None, ux=None, uy=None, uz=None):
        shp = self.shape
        r, a, b, c = self._dev(rho, shp), self._dev(ux, shp), self._dev(uy, shp), self._dev(uz, shp)
        with self._torch.cuda.device(self.device):
            _check(self.lib.glbm_init_fields3(self._h, self._ptr(r), self._ptr(a), self._ptr(b), self._ptr(c)),
                   "glbm_init_fields3")
        self._keep = [r, a, b, c]

    def init_populations(self, f0):
        t = self._dev(f0, (self.Q,) + self.shape)
        with self._torch.cuda.device(self.device):
            _check(self.lib.glbm_init_populations(self._h, self._ptr(t)), "glbm_init_populations")
        self._keep = [t]

    def step(self, n: int = 1):
        with self._torch.cuda.device(self.device):
            _check(self.lib.glbm_step(self._h, int(n)), "glbm_step")

    def moments(self, which=None) -> dict:
        """rho, ux, uy, T, pxy (and uz in three dimensions) of f(t), shaped
        like the lattice ([nz][ny][nx] or [ny][nx])."""
        torch = self._torch
        if which is None:
            which = ("rho", "ux", "uy", "uz", "T", "pxy") if self.dims == 3 else ("rho", "ux", "uy", "T", "pxy")
        out = {k: torch.empty(self.shape, dtype=torch.float32, device=self.device) for k in which}
        ptrs = [self._ptr(out.get(k)) for k in ("rho", "ux", "uy", "uz", "T", "pxy")]
        with torch.cuda.device(self.device):
            _check(self.lib.glbm_moments3(self._h, *ptrs), "glbm_moments3")
        return out

    def populations(self):
        torch = self._torch
        out = torch.empty((self.Q,) + self.shape, dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            _check(self.lib.glbm_get_populations(self._h, self._ptr(out)), "glbm_get_populations")
        return out

    def stats(self, static: bool = False) -> dict:
        """FP64 diagnostics; ``health`` is "ok", "nonfinite" (some node blew
        up) or "positivity" (some node left the positivity domain).  static:
        through glbm_stats_static (no device allocation; calls on one GPU must
        not overlap)."""
        s = Stats()
        fn = self.lib.glbm_stats_static if static else self.lib.glbm_stats
        with self._torch.cuda.device(self.device):
            rc = fn(self._h, ctypes.byref(s))
        if rc not in HEALTH:
            _check(rc, "glbm_stats")
        return {
            "health": HEALTH[rc], "nonfinite_nodes": s.nonfinite_nodes,
            "time": s.time, "mass": s.mass, "momentum_x": s.momentum_x, "momentum_y": s.momentum_y,
            "energy_post": s.energy_post, "residual": s.residual,
            "wall_mass_bottom": s.wall_mass[0], "wall_mass_top": s.wall_mass[1],
            "wall_momentum_bottom": s.wall_momentum[0], "wall_momentum_top": s.wall_momentum[1],
            "nonpositive_nodes": s.nonpositive_nodes, "momentum_z": s.momentum_z,
        }

    def info(self) -> dict:
        tau, om = ctypes.c_double(), ctypes.c_double()
        q, t = ctypes.c_int32(), ctypes.c_int64()
        _check(self.lib.glbm_info(self._h, ctypes.byref(tau), ctypes.byref(om), ctypes.byref(q), ctypes.byref(t)),
               "glbm_info")
        return {"tau": tau.value, "omega": om.value, "nvel": q.value, "time": t.value}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _check(self.lib.glbm_destroy(h), "glbm_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many solvers stepped together (glbm_batch_*): one launch per kernel
    variant and step over a tile table, optionally replayed from a captured
    HIP graph of ``graph_steps`` steps.  Members keep their own buffers and
    can be observed while in the batch; ``close()`` hands them back."""

    def __init__(self, solvers, tile_nodes: int = 256, order: str = "member", graph_steps: int = 0, stream=None,
                 resident_nodes: int = 0, streams: int = 1):
        import torch

        if not solvers:
            raise GlbmError("a batch needs at least one solver")
        self._torch = torch
        self.lib = load()
        self.solvers = list(solvers)
        self.device = self.solvers[0].device
        self.stream = stream if stream is not None else self.solvers[0].stream
        self.options = {"tile_nodes": int(tile_nodes), "order": order, "graph_steps": int(graph_steps),
                        "resident_nodes": int(resident_nodes), "streams": int(streams)}
        opt = BatchOptions(int(tile_nodes), ORDER[order], int(graph_steps), int(resident_nodes), int(streams))
        arr = (ctypes.c_void_p * len(self.solvers))(*[s._h.value for s in self.solvers])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.glbm_batch_create(arr, len(self.solvers), ctypes.byref(opt),
                                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                   "glbm_batch_create")
        self._h = h

    def step(self, n: int = 1):
        with self._torch.cuda.device(self.device):
            _check(self.lib.glbm_batch_step(self._h, int(n)), "glbm_batch_step")

    def update(self, solvers):
        """Replace the member set (solvers join and leave between steps)."""
        solvers = list(solvers)
        arr = (ctypes.c_void_p * max(1, len(solvers)))(*[s._h.value for s in solvers])
        with self._torch.cuda.device(self.device):
            _check(self.lib.glbm_batch_update(self._h, arr, len(solvers)), "glbm_batch_update")
        self.solvers = solvers

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.glbm_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def bandwidth_probe(mode: str, nbytes: int, reps: int = 20, blocks: int = 4096, device=None) -> dict:
    """Time the library's streaming kernels (glbm_bandwidth_probe): "copy"
    (nbytes read + nbytes written), "read" or "write", `reps` launches on the
    current stream; returns the average launch time and the rate."""
    import torch

    lib = load()
    code = {"copy": 0, "read": 1, "write": 2}[mode]
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty(nbytes // 4 if mode != "read" else 4, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    sp = ctypes.c_void_p(stream.cuda_stream)

    def launch():
        _check(lib.glbm_bandwidth_probe(code, src.data_ptr(), dst.data_ptr(), nbytes, blocks, sp),
               "glbm_bandwidth_probe")

    launch()
    torch.cuda.synchronize(dev)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        launch()
    stop.record(stream)
    torch.cuda.synchronize(dev)
    sec = start.elapsed_time(stop) / 1e3 / reps
    moved = 2 * nbytes if mode == "copy" else nbytes
    return {"mode": mode, "bytes": nbytes, "blocks": blocks, "us": round(sec * 1e6, 1),
            "GBs": round(moved / sec / 1e9, 1)}


def solver_for(workload, device=None, stream=None) -> Solver:
    return Solver(config_from_workload(workload), device=device, stream=stream)
