"""Host-side logic on the CPU: the seeded input recipes of the batched sweep
and the served mix, lane assignment and admission of the server, latency
summaries, the autotuner's candidate set.  No GPU is touched."""
import math

import numpy as np
import pytest

from paper_1905_04597_amd import batching, serving
from paper_1905_04597_amd import workloads as wl


# ------------------------------------------------------------ recipes
def test_sweep_recipe():
    ws = wl.sweep_workloads()
    assert len(ws) == 512
    kinds = [w.name.split("_")[0] for w in ws]
    assert set(kinds) == {"couette", "poiseuille"}
    assert 0.4 < kinds.count("couette") / 512 < 0.6
    for w in ws:
        assert w.dims == 2 and w.nx == 4 and 32 <= w.ny <= 1024 and 2 <= w.level_x == w.level_y <= 6
        assert w.bc_y == "wall" and w.steps == 2000 and w.storage == "f32_shifted"
        assert 1e-3 <= w.kn <= 10
        cs = math.sqrt(w.level_y / 3.0)
        if w.name.startswith("couette"):
            assert w.g == 0 and w.wall_u[0] == -w.wall_u[1] and 0.01 * cs <= w.wall_u[1] <= 0.1 * cs
        else:
            # g = 8 nu U / H^2 with U in [0.01, 0.1] c_s, nu = theta tau, tau = Kn H / sqrt(2 theta)
            theta, H = w.level_y / 3.0, float(w.ny)
            nu = theta * w.kn * H / math.sqrt(2 * theta)
            U = w.g * H * H / (8 * nu)
            assert w.wall_u == (0.0, 0.0) and 0.01 * cs * (1 - 1e-12) <= U <= 0.1 * cs * (1 + 1e-12)
    # the same draw every time
    again = wl.sweep_workloads()
    assert [(w.ny, w.level_y, w.kn, w.g, w.wall_u) for w in ws] == [(w.ny, w.level_y, w.kn, w.g, w.wall_u)
                                                                     for w in again]
    assert sum(w.nodes for w in ws) == 1071044  # the nodes the batched bench reports


def test_served_recipe():
    reqs = wl.served_requests()
    n = len(reqs)
    # Poisson arrivals at 200/s over 12 s: 2400 +- 3 sigma
    assert abs(n - 2400) < 3 * math.sqrt(2400)
    t = np.array([a for a, _ in reqs])
    assert np.all(np.diff(t) > 0) and 0 < t[0] and t[-1] < 12.0
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert gaps.mean() == pytest.approx(1 / 200.0, rel=0.06)
    kinds = [w.name.split("_")[0] for _, w in reqs]
    for k in ("sod", "couette", "poiseuille"):
        assert 0.28 < kinds.count(k) / n < 0.39
    storages = [w.storage for _, w in reqs]
    assert set(storages) == {"f32_shifted", "bf16_shifted_sr"}
    for _, w in reqs:
        assert 1 <= w.level_x <= 7
        if w.dims == 1:
            assert w.bc_x == "eq_ends" and 500 <= w.nx <= 20000 and w.steps == 1000
        else:
            assert w.bc_y == "wall" and 32 <= w.ny <= 2048 and 4 <= w.nx <= 2048 and w.steps == 200
    # arrivals and parameters come from separate seeds
    other = wl.served_requests(arrival_seed=7)
    assert [w.level_x for _, w in other[:50]] == [w.level_x for _, w in reqs[:50]]
    assert [a for a, _ in other[:50]] != [a for a, _ in reqs[:50]]


# ------------------------------------------------------------- server
def test_step_bytes():
    w = wl.poiseuille(nx=4096, ny=1024, level=5, storage="f32_shifted")
    assert serving.step_bytes(w) == 2 * 4096 * 1024 * 121 * 4
    w.storage = "bf16_shifted_sr"
    assert serving.step_bytes(w) == 2 * 4096 * 1024 * 121 * 2


def test_lanes_by_size_and_variant():
    light, nl = 64 << 20, 3
    big = wl.poiseuille(nx=2048, ny=2048, level=5, storage="f32_shifted")
    assert serving.step_bytes(big) >= light and serving.lane_of(big, light, nl) == nl
    # the same kernel variant goes to the same light lane, whatever its size
    a = wl.couette(0.1, ny=64, nx=4, level=3, storage="f32_shifted")
    b = wl.couette(1.0, ny=300, nx=40, level=3, storage="f32_shifted")
    assert serving.lane_of(a, light, nl) == serving.lane_of(b, light, nl) < nl
    # the served mix spreads over every light lane and the heavy one
    lanes = [serving.lane_of(w, light, nl) for _, w in wl.served_requests()]
    assert set(lanes) == {0, 1, 2, 3}


def test_admission_is_first_come_first_served_within_budget_and_slots():
    GB = 1e9
    assert serving.admissible([10 * GB, 20 * GB, 30 * GB], 0.0, 200 * GB, 10) == 3
    # the budget stops at the first request that does not fit: no overtaking
    assert serving.admissible([10 * GB, 190 * GB, 1 * GB], 5 * GB, 200 * GB, 10) == 1
    assert serving.admissible([10 * GB, 10 * GB], 195 * GB, 200 * GB, 10) == 0
    # slots
    assert serving.admissible([1 * GB] * 5, 0.0, 200 * GB, 2) == 2
    assert serving.admissible([], 0.0, 200 * GB, 2) == 0
    assert serving.admissible([1 * GB], 0.0, 200 * GB, 0) == 0
    # a request exactly filling the budget is admitted
    assert serving.admissible([50 * GB], 150 * GB, 200 * GB, 1) == 1


def test_summary_of_latencies():
    w = wl.couette(0.1, ny=32, nx=4, level=1)
    reqs = []
    for i in range(200):
        r = serving.Request(i, arrival=1.0 + i * 0.05, workload=w, steps=10)
        r.finished = r.arrival + (i % 100 + 1) * 0.01   # latencies 0.01 .. 1.00, twice
        reqs.append(r)
    reqs[-1].finished = None  # not finished
    s = serving.summarize(reqs, window=(2.0, 12.0))
    meas = [r for r in reqs if 2.0 <= r.arrival < 12.0]
    assert s["requests"] == len(meas) and s["completed"] == len(meas) - 1
    lat = sorted(r.latency for r in meas if r.finished is not None)
    assert s["latency_p50_s"] == pytest.approx(np.percentile(lat, 50), abs=1e-4)
    assert s["latency_p99_s"] == pytest.approx(np.percentile(lat, 99), abs=1e-4)
    assert s["latency_max_s"] == pytest.approx(max(lat), abs=1e-4)
    span = max(r.finished for r in meas if r.finished is not None) - 2.0
    assert s["solves_per_s"] == pytest.approx(s["completed"] / span, abs=0.01)
    assert s["node_steps"] == s["completed"] * w.nodes * 10


def test_autotuner_candidates():
    c = batching.candidates()
    assert len(c) == 3 * 3 * 2 * 2 * 3
    assert len({tuple(sorted(d.items())) for d in c}) == len(c)
    assert all(d["tile_nodes"] in (64, 128, 256) for d in c)
