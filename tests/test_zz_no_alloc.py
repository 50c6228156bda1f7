"""glbm_stats_static, the statistics entry point that allocates nothing (for
callers that cannot allocate: graph capture, serving loops), against
glbm_stats on the same solvers: two calls in a row on one GPU, the second on
a smaller lattice, each equal field by field (same kernels, same block
count: the sums are bitwise the same)."""
import ctypes
import math

import numpy as np
import pytest

from paper_1905_04597_amd import glbm
from paper_1905_04597_amd import workloads as wl

pytestmark = pytest.mark.gpu

FIELDS = [name for name, _ in glbm.Stats._fields_]


def _values(s):
    out = {}
    for name in FIELDS:
        v = getattr(s, name)
        out[name] = list(v) if hasattr(v, "__len__") else v
    return out


def _same(a, b):
    if isinstance(a, list):
        return all(_same(x, y) for x, y in zip(a, b))
    if isinstance(a, float) and math.isnan(a):
        return isinstance(b, float) and math.isnan(b)
    return a == b


def _both(solver):
    lib = glbm.load()
    ref, got = glbm.Stats(), glbm.Stats()
    rc_ref = lib.glbm_stats(solver._h, ctypes.byref(ref))
    rc_got = lib.glbm_stats_static(solver._h, ctypes.byref(got))
    return rc_ref, _values(ref), rc_got, _values(got)


@pytest.mark.parametrize("first", [(1024, 1024), (300, 7)], ids=["strided", "small"])
def test_static_stats_equal_allocating_stats(first):
    import torch

    # first call: a lattice of (nx, ny) (1024 x 1024 needs more blocks than the
    # statistics launch takes, so the blocks stride); second: a smaller one
    sizes = [first, (37, 21)]
    for k, (nx, ny) in enumerate(sizes):
        cfg = glbm.make_config(2, 2, 2, nx, ny, tau=0.8, bc_y="wall", wall_u=(-0.03, 0.02), g=1e-5,
                               storage="f32_shifted")
        s = glbm.Solver(cfg)
        rho, ux, uy = wl.random_fields(5 + k, nx, ny, rho_amp=0.05, u_amp=0.05, dims=2)
        s.init_fields(rho, ux, uy)
        s.step(3)
        torch.cuda.synchronize()
        rc_ref, ref, rc_got, got = _both(s)
        print("\n[no-alloc] call %d on %dx%d: status %d/%d mass %.15g / %.15g"
              % (k, nx, ny, rc_ref, rc_got, ref["mass"], got["mass"]), flush=True)
        assert rc_got == rc_ref == glbm.OK
        for name in FIELDS:
            assert _same(ref[name], got[name]), (name, ref[name], got[name])
        assert got["time"] == 3 and got["mass"] > 0.9 * nx * ny
        s.close()


def test_static_stats_report_failure_like_the_allocating_one():
    cfg = glbm.make_config(2, 2, 2, 40, 12, tau=0.8, storage="f32_shifted")
    s = glbm.Solver(cfg)
    f0 = wl.random_populations(3, 25, 40, 12)
    f0[7, 5, 6] = np.nan
    s.init_populations(f0)
    s.step(1)
    rc_ref, ref, rc_got, got = _both(s)
    assert rc_ref == rc_got == glbm.ERR_NONFINITE
    assert got["nonfinite_nodes"] == ref["nonfinite_nodes"] > 0
    s.close()
