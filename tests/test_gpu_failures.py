"""Failure detection (the statuses of glbm_stats and the server's retirement
of a blown-up request), driven by data only: a NaN plane of initial
populations, velocities outside the positivity domain of section 3, and a
Sod tube at a viscosity where the oracle itself breaks down.  The counts are
compared with the oracle's own (tests/test_oracle_diagnostics.py pins them).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1905_04597_amd import glbm
from paper_1905_04597_amd import serving
from paper_1905_04597_amd import workloads as wl
from tests.gpu_common import make_pair

pytestmark = pytest.mark.gpu


def _nan_populations(Q, nx, ny, nodes_xy, seed=11):
    f0 = wl.random_populations(seed, Q, nx, ny)
    for (x, y) in nodes_xy:
        f0[Q // 3, y, x] = np.nan
    return f0


def test_nan_plane_is_counted_and_reported():
    params = dict(dims=2, level_x=2, level_y=2, nx=37, ny=21, tau=0.8, bc_y="wall", wall_u=(-0.02, 0.03), g=1e-5)
    bad = [(3, 4), (30, 10), (36, 20)]
    f0 = _nan_populations(25, 37, 21, bad)
    for storage in ("f32_shifted", "bf16_shifted_sr"):
        orc, gpu = make_pair(params, storage)
        orc.init_populations(f0.astype(np.float64))
        gpu.init_populations(f0)
        print("\n[failures] nan plane storage=%s" % storage, flush=True)
        for steps in (0, 1, 3):
            if steps:
                orc.step(steps - orc.time)
                gpu.step(steps - gpu.info()["time"])
            so, sg = orc.stats(), gpu.stats()
            print("[failures] t=%d gpu nonfinite %d health %s, oracle nonfinite %d"
                  % (steps, sg["nonfinite_nodes"], sg["health"], so["nonfinite_nodes"]), flush=True)
            assert sg["health"] == "nonfinite"
            assert sg["nonfinite_nodes"] == so["nonfinite_nodes"] > 0
        assert so["nonfinite_nodes"] > len(bad)  # the NaN spreads with the streaming
        # the C status itself
        s = glbm.Stats()
        assert gpu.lib.glbm_stats(gpu._h, s) == glbm.ERR_NONFINITE
        assert b"non-finite" in gpu.lib.glbm_last_error()
        gpu.close()


def test_positivity_domain_count_matches_the_oracle():
    # u_x above sqrt(2 N theta0) = sqrt(2 N^2 / 3) on some nodes (N = 2: 1.633)
    nx, ny = 40, 12
    ux = np.zeros((ny, nx), np.float32)
    ux[2, 5] = 1.7
    ux[7, 30] = -1.66
    ux[9, 9] = 1.6  # inside
    params = dict(dims=2, level_x=2, level_y=2, nx=nx, ny=ny, tau=0.8)
    orc, gpu = make_pair(params, "f32_shifted")
    rho = np.ones((ny, nx), np.float32)
    orc.init_fields(rho.astype(np.float64), ux.astype(np.float64), np.zeros((ny, nx)))
    gpu.init_fields(rho, ux, np.zeros_like(ux))
    so, sg = orc.stats(), gpu.stats()
    print("\n[failures] positivity gpu %d (%s) oracle %d" % (sg["nonpositive_nodes"], sg["health"],
                                                             so["nonpositive_nodes"]), flush=True)
    assert so["nonpositive_nodes"] == 2
    assert sg["nonpositive_nodes"] == so["nonpositive_nodes"]
    assert sg["health"] == "positivity" and sg["nonfinite_nodes"] == 0


def test_sod_breakdown_is_detected_like_the_oracle():
    """The Sod tube of section 5.1 (density 4 | 1, 800 nodes) on D1Q3 at a
    viscosity below its stable range.  After 100 steps the oracle has
    negative densities (a breakdown) and nodes outside the positivity domain:
    the GPU flags the state too.  By 400 steps the oracle's densities exceed
    the FP32 range (FP64 still holds them), so an FP32 solver has overflowed:
    the GPU reports non-finite nodes."""
    nodes, nu = 800, 0.0005
    rho0 = np.where((np.arange(nodes) + 0.5) / nodes <= 0.5, 4.0, 1.0)
    orc = oracle.OracleSolver(1, 1, 0, nodes, 1, tau=nu, bc_x=oracle.BC_EQ_ENDS, end_rho=(4.0, 1.0))
    orc.init_fields(rho0)
    cfg = glbm.make_config(1, 1, 0, nodes, 1, tau=nu, bc_x="eq_ends", end_rho=(4.0, 1.0), storage="f32_shifted")
    gpu = glbm.Solver(cfg)
    gpu.init_fields(rho0.astype(np.float32), np.zeros(nodes, np.float32))
    for steps in (100, 400):
        orc.step(steps - orc.time)
        gpu.step(steps - gpu.info()["time"])
        so, sg = orc.stats(), gpu.stats()
        rmax = float(np.max(np.abs(orc.moments()["rho"])))
        print("\n[failures] sod D1Q3 nu=%g t=%d: oracle nonpositive %d max|rho| %.1e; gpu %s nonfinite %d "
              "nonpositive %d" % (nu, steps, so["nonpositive_nodes"], rmax, sg["health"], sg["nonfinite_nodes"],
                                  sg["nonpositive_nodes"]), flush=True)
        assert so["nonpositive_nodes"] > 0 and sg["health"] != "ok"
    assert rmax > float(np.finfo(np.float32).max)
    assert sg["health"] == "nonfinite" and sg["nonfinite_nodes"] > 0


def test_server_retires_a_blown_up_request_and_the_others_are_unchanged():
    U = 0.05 * math.sqrt(2 / 3.0)
    good = [wl.couette(0.1, ny=24, nx=8, level=2, steps=60, storage="f32_shifted"),
            wl.poiseuille(nx=16, ny=20, level=2, kn=0.2, g=1e-5, steps=40, storage="bf16_shifted_sr"),
            wl.sod(nodes=600, level=3, steps=80, storage="f32_shifted")]
    bad_w = wl.Workload("nan", 2, 2, 2, 12, 16, tau=0.9, bc_y="wall", wall_u=(-U, U), steps=60,
                        storage="f32_shifted")
    f0 = _nan_populations(25, 12, 16, [(4, 8)])
    arrivals = [(0.0, good[0]), (0.0, bad_w, f0), (0.001, good[1]), (0.002, good[2])]
    srv = serving.Server(keep_results=True, check_every=1, chunks=(10, 10))
    reqs = srv.run(arrivals, max_seconds=60)
    by = {r.rid: r for r in reqs}
    print("\n[failures] server health %s" % [(r.rid, r.health, r.failed) for r in reqs], flush=True)
    assert by[1].failed and by[1].health == "nonfinite" and by[1].result is None
    # retired at the first check, before its step budget ran out
    assert by[1].finished is not None
    for rid, w in ((0, good[0]), (2, good[1]), (3, good[2])):
        r = by[rid]
        assert r.health == "ok" and r.result is not None
        alone = serving.solve_alone(w, w.steps)
        for k in alone:
            assert np.array_equal(alone[k].cpu().numpy(), r.result[k].cpu().numpy()), (rid, k)
