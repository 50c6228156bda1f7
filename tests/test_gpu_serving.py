"""The continuous-batching server (paper_1905_04597_amd.serving).

Requests of the served mix (Sod, Couette and Poiseuille solves of different
sizes, levels, Knudsen numbers and storages) arrive over time, are admitted
into two lanes as slots and the device-memory budget allow, and leave when
their step budget is spent.  Each result must equal the same solve run alone
(one lattice, one launch per step) bitwise: a batched lattice runs exactly
the single-lattice kernel code.
"""
import pytest

from paper_1905_04597_amd import serving
from paper_1905_04597_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _same(a, b) -> bool:
    import torch

    for k in ("rho", "ux", "uy", "T", "pxy"):
        x, y = a[k], b[k]
        if not bool(((x == y) | (torch.isnan(x) & torch.isnan(y))).all()):
            return False
    return True


def _small(arrivals, max_pop_bytes):
    return [(t, w) for t, w in arrivals if serving.step_bytes(w) <= max_pop_bytes]


def test_served_results_equal_alone():
    arrivals = wl.served_requests(duration=0.25)
    print("\n[serving] %d requests over 0.25 s" % len(arrivals), flush=True)
    srv = serving.Server(keep_results=True, chunks=(50, 20))
    reqs = srv.run(arrivals, max_seconds=60)
    assert all(r.finished is not None for r in reqs)
    assert srv.in_use == 0
    lat = sorted(r.latency for r in reqs)
    print("[serving] completed %d, lanes %s, latency p50 %.4f s max %.4f s, chunks %s"
          % (len(reqs), [sum(r.lane == i for r in reqs) for i in range(len(srv.lanes))], lat[len(lat) // 2], lat[-1],
             [l.chunks for l in srv.lanes]), flush=True)
    for r in reqs:
        alone = serving.solve_alone(r.workload, r.steps)
        assert _same(r.result, alone), (r.rid, r.workload)


def test_budget_admission_holds_requests_back():
    """A budget that fits only a few requests at a time: requests wait for
    memory, the budget is never exceeded and every result still equals the
    solve run alone."""
    arrivals = _small(wl.served_requests(duration=0.15), 16 << 20)
    budget = 3 * max(2 * serving.glbm.population_bytes(serving.glbm.config_from_workload(w)) for _, w in arrivals)
    srv = serving.Server(hbm_budget=budget, keep_results=True, chunks=(40, 20))
    reqs = srv.run(arrivals, max_seconds=60)
    print("\n[serving] %d requests, budget %d bytes, peak %d" % (len(reqs), budget, srv.peak_in_use), flush=True)
    assert srv.peak_in_use <= budget
    assert all(r.finished is not None for r in reqs)
    waited = sum(r.admitted - r.arrival > 1e-3 for r in reqs)
    print("[serving] %d requests waited for memory" % waited, flush=True)
    for r in reqs:
        assert _same(r.result, serving.solve_alone(r.workload, r.steps)), r.rid


def test_per_solve_loop_runs_every_request():
    arrivals = _small(wl.served_requests(duration=0.05), 16 << 20)
    reqs = serving.serve_per_solve(arrivals, max_seconds=60)
    assert all(r.finished is not None and r.finished >= r.arrival for r in reqs)
    summ = serving.summarize(reqs, window=(0.0, 0.05))
    assert summ["completed"] == len(arrivals)
