"""Benchmark of the fused stream-collide step on one MI355X.

Workload (default): force-driven Poiseuille channel, tensor-product
G-D2Q(11x11) (level N = 5 per axis, k = 4, 121 velocities), 4096 x 1024
nodes, diffuse walls at rest, g = 1e-5, Kn = 0.1, FP32 populations stored as
deviations from the rest state (the FP32 path that meets 1e-5); inputs are
resident in HBM before the timed region.  One "step" is one time step of the
whole lattice (one launch of the fused kernel).

Prints ONE JSON line: GLUPS (1e9 node updates per second), the roofline of
the step kernel (algorithmic bytes 2 Q s per node update over the average
launch duration, against the 8 TB/s HBM peak), a per-level sweep, the batched
channel sweep (512 uneven instances, batched vs the per-solve loop), the
served mix (continuous batching vs the per-solve loop, p50/p99 latency) and
the FP64 oracle timed on the host cores over a bounded sample.

    python bench.py [--steps K] [--warmup W] [--storage f32_shifted|bf16_shifted_sr|...]
                    [--no-sweep] [--no-batched] [--no-served] [--no-cpu-baseline]
                    [--batched-only] [--served-only]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
ELEM_BYTES = {"f32": 4, "f32_shifted": 4, "bf16_shifted": 2, "bf16_shifted_sr": 2}
DTYPE = {"f32": "f32", "f32_shifted": "f32", "bf16_shifted": "bf16", "bf16_shifted_sr": "bf16"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_poiseuille_d2q121_4096x1024.json")


def kernel_source_hash() -> str:
    from paper_1905_04597_amd import profiling

    return profiling.kernel_source_hash()


def time_steps(solver, steps: int, warmup: int):
    """Warm up, then time exactly `steps` launches with events on the solver's stream."""
    import torch

    solver.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(solver.stream)
    t0 = time.perf_counter()
    solver.step(steps)
    stop.record(solver.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / 1e3, wall


def run_gpu(level: int, nx: int, ny: int, storage: str, steps: int, warmup: int, lattice: str = "odd"):
    """lattice: "odd" G-D1Q(2N+1) on both axes, "even" G-D1Q(2N+2) on both,
    "mixed_even" D1Q3 along the channel x G-D1Q(2N+2) across it."""
    from paper_1905_04597_amd import glbm
    from paper_1905_04597_amd import workloads as wl

    def make(rows):
        w = wl.poiseuille(nx=nx, ny=rows, level=level, storage=storage)
        if lattice == "even":
            w.even_x = w.even_y = True
        elif lattice == "mixed_even":
            w.level_x, w.even_y = 1, True
        return w

    w = make(ny)
    # a population buffer stays below 4 GiB (32-bit offsets): G-D2Q256 in
    # FP32 at 4096 x 1024 would need exactly 4 GiB, so it runs one row fewer
    rows_max = ((1 << 32) - 1) // (w.nvel * ELEM_BYTES[storage] * nx)
    if ny > rows_max:
        ny = rows_max
        w = make(ny)
    s = glbm.solver_for(w)
    s.init_fields()
    gpu_s, wall_s = time_steps(s, steps, warmup)
    nodes = nx * ny
    Q = w.nvel
    per_step = gpu_s / steps
    algo_bytes = 2 * Q * ELEM_BYTES[storage] * nodes
    out = {
        "level": level, "k": level - 1, "Q": Q, "ny": ny, "glups": nodes * steps / gpu_s / 1e9,
        "ms_per_step": per_step * 1e3, "achieved_GBs": algo_bytes / per_step / 1e9,
        "bytes_per_launch": algo_bytes, "wall_s": wall_s,
    }
    st = s.stats()
    out["mass_drift_rel"] = abs(st["mass"] - nodes) / nodes
    s.close()
    return out


# Three-dimensional sweep lines: D3Q27, G-D3Q125, G-D3Q343 and the channels
# D1Q3 x G-D1Q(2N+1) x D1Q3 and D1Q3 x G-D1Q(2N+2) x D1Q3, N = 2..7.
SWEEP_3D = [((1, 1, 1), False, (256, 256, 128)), ((2, 2, 2), False, (128, 128, 128)),
            ((3, 3, 3), False, (128, 128, 128))] + [
    ((1, n, 1), ev, (256, 128, 128)) for ev in (False, True) for n in range(2, 8)]


def run_gpu3(levels, even_y: bool, nx: int, ny: int, nz: int, storage: str, steps: int, warmup: int):
    """A three-dimensional lattice (periodic x, z; walls across y), force-driven
    from rest, timed like run_gpu."""
    from paper_1905_04597_amd import glbm

    lx, ly, lz = levels
    cfg = glbm.make_config(3, lx, ly, nx, ny, kn=0.1, bc_y="wall", g=1e-5, storage=storage, even_y=even_y,
                           level_z=lz, nz=nz)
    s = glbm.Solver(cfg)
    s.init_fields()
    gpu_s, _ = time_steps(s, steps, warmup)
    nodes = nx * ny * nz
    per_step = gpu_s / steps
    algo = 2 * s.Q * ELEM_BYTES[storage] * nodes
    s.close()
    return {"lattice": "3d", "levels": list(levels), "even_y": even_y, "shape": [nx, ny, nz], "Q": s.Q,
            "glups": round(nodes * steps / gpu_s / 1e9, 4), "ms_per_step": round(per_step * 1e3, 4),
            "achieved_GBs": round(algo / per_step / 1e9, 1), "frac": round(algo / per_step / 1e9 / PEAK_HBM_GBS, 4)}


def bandwidth_ceiling(nbytes: int = 2 << 30, reps: int = 10) -> dict:
    """The library's hand-written streaming kernels (glbm_bandwidth_probe:
    16-byte non-temporal accesses, grid-stride) on buffers of the step's
    size: copy (read + write 1:1, the step's own mix), read only, write
    only; the best of three grid sizes each."""
    from paper_1905_04597_amd import glbm

    out = {}
    for mode in ("copy", "read", "write"):
        best = max((glbm.bandwidth_probe(mode, nbytes, reps=reps, blocks=b) for b in (2048, 8192, 32768)),
                   key=lambda r: r["GBs"])
        out[mode + "_GBs"] = best["GBs"]
        out[mode + "_blocks"] = best["blocks"]
    out["bytes"] = nbytes
    return out


def copy_probe(nbytes: int = 2 << 30, reps: int = 10):
    """PyTorch's device copy of known size (for comparison with the
    library's own copy kernel)."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        b.copy_(a)
    stop.record()
    torch.cuda.synchronize()
    sec = start.elapsed_time(stop) / 1e3 / reps
    return {"bytes_each_way": nbytes, "reps": reps, "GBs": round(2 * nbytes / sec / 1e9, 1)}


def run_batched(count: int = 512, steps: int = 2000, storage: str = "f32_shifted", loop_steps: int = 2000,
                tune_steps: int = 64):
    """The batched channel sweep: `count` uneven Couette / Poiseuille
    instances (Nx = 4, Ny 32..1024, levels 2..6), `steps` steps each.

    The schedule is autotuned on scratch lattices; the tuned batch is timed
    over all `steps` steps; the plain per-solve loop (each instance alone,
    one launch per step, one instance after the other on one stream) is
    timed over `loop_steps` steps per instance on fresh lattices.  When the
    step counts agree, every instance's populations are compared bitwise
    between the two."""
    import torch
    from paper_1905_04597_amd import batching, glbm
    from paper_1905_04597_amd import workloads as wl

    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    ws = wl.sweep_workloads(count, steps=steps, storage=storage)
    cfgs = [glbm.config_from_workload(w) for w in ws]
    nodes = sum(w.nodes for w in ws)
    pops = sum(w.nodes * w.nvel for w in ws)
    t0 = time.perf_counter()
    best, table = batching.autotune(cfgs, steps=tune_steps)
    tune_s = time.perf_counter() - t0

    batched = [glbm.Solver(c) for c in cfgs]
    for s in batched:
        s.init_fields()
    torch.cuda.synchronize()
    b = glbm.Batch(batched, **best)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    b.step(steps)
    stop.record()
    torch.cuda.synchronize()
    batch_s = start.elapsed_time(stop) / 1e3
    b.close()

    loop = [glbm.Solver(c) for c in cfgs]
    for s in loop:
        s.init_fields()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(count + 1)]
    ev[0].record()
    for i, s in enumerate(loop):
        s.step(loop_steps)
        ev[i + 1].record()
    torch.cuda.synchronize()
    done = [ev[0].elapsed_time(e) / 1e3 for e in ev[1:]]
    loop_s = done[-1]

    equal = None
    if loop_steps == steps:
        equal = all(torch.equal(a.populations(), c.populations()) for a, c in zip(batched, loop))
    for s in batched + loop:
        s.close()
    bytes_step = sum(2 * w.nodes * w.nvel * ELEM_BYTES[storage] for w in ws)
    per_solve = loop_s / loop_steps * steps
    done_sorted = sorted(d / loop_steps * steps for d in done)
    return {
        "workload": "%d Couette/Poiseuille channels, Nx=4, Ny~U{32..1024}, level~U{2..6}, log10 Kn~U[-3,1], "
                    "speed~U[0.01,0.1] c_s, %d steps each, seed 190504597" % (count, steps),
        "storage": storage, "instances": count, "nodes": nodes, "populations": pops,
        "schedule": best, "autotune_s": round(tune_s, 2),
        "autotune_us_per_step": {"%(tile_nodes)d/%(order)s/g%(graph_steps)d/r%(resident_nodes)d/s%(streams)d" % o: round(sec * 1e6, 1)
                                 for o, sec in table},
        "batched": {"solves_per_s": round(count / batch_s, 2), "seconds": round(batch_s, 4),
                    "glups": round(nodes * steps / batch_s / 1e9, 3),
                    "achieved_GBs": round(bytes_step * steps / batch_s / 1e9, 1),
                    "latency_p50_s": round(batch_s, 4), "latency_p99_s": round(batch_s, 4)},
        "per_solve_loop": {"solves_per_s": round(count / per_solve, 2), "seconds": round(per_solve, 4),
                           "measured_steps": loop_steps,
                           "glups": round(nodes * steps / per_solve / 1e9, 3),
                           "latency_p50_s": round(done_sorted[len(done_sorted) // 2], 4),
                           "latency_p99_s": round(done_sorted[min(count - 1, int(0.99 * count))], 4)},
        "speedup": round(per_solve / batch_s, 2),
        "bitwise_equal": equal,
    }


def run_solves():
    """Time per solve of the Sod tube (D1Q7, 2000 nodes, Kn = 0.01, 1000 steps)
    and the Couette channels (G-D2Q49, 4 x 256, Kn 0.01 / 0.1 / 1 / 10, run for
    the number of steps at which the FP64 reference reached a residual of
    1e-10: 15300 / 2600 / 5000 / 40500): one launch per step; the same solve
    as a one-member batch of 64-node tiles replayed from 100-step HIP graphs;
    and as a one-member resident batch (one workgroup, every step of the solve
    in one launch).  All give bitwise the same populations (checked)."""
    import numpy as np
    import torch
    from paper_1905_04597_amd import glbm
    from paper_1905_04597_amd import workloads as wl

    cases = [("sod_d1q7_2000_kn0.01", wl.sod(2000, 3, 0.01, 1000, storage="f32_shifted"), 1000)]
    for kn, steps in ((0.01, 15300), (0.1, 2600), (1.0, 5000), (10.0, 40500)):
        cases.append(("couette_d2q49_4x256_kn%g" % kn, wl.couette(kn, storage="f32_shifted"), steps))
    out = {}
    for name, w, steps in cases:
        times = {}
        pops = []
        for mode in ("per_step_launch", "graph", "resident"):
            s = glbm.solver_for(w)
            if w.init == "sod":
                rho = wl.sod_density(w.nx, *w.end_rho)
                s.init_fields(rho, np.zeros_like(rho))
            else:
                s.init_fields()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "resident":
                with glbm.Batch([s], resident_nodes=w.nodes) as b:
                    b.step(steps)
            elif mode == "graph":
                with glbm.Batch([s], tile_nodes=64, graph_steps=100) as b:
                    b.step(steps)
            else:
                s.step(steps)
            torch.cuda.synchronize()
            times[mode] = time.perf_counter() - t0
            pops.append(s.populations())
            s.close()
        out[name] = {"steps": steps, "nodes": w.nodes, "velocities": w.nvel,
                     "ms_per_solve": {k: round(v * 1e3, 2) for k, v in times.items()},
                     "bitwise_equal": all(bool(torch.equal(pops[0], p)) for p in pops[1:])}
    return out


def _same_moments(a, b) -> bool:
    import torch

    return all(bool(((a[k] == b[k]) | (torch.isnan(a[k]) & torch.isnan(b[k]))).all())
               for k in ("rho", "ux", "uy", "T", "pxy"))


def run_served(duration: float = 12.0, warm: float = 2.0, sample: int = 16, loop_max: float = 90.0):
    """The served mix: Poisson arrivals at 200 requests/s (seeds 1905 / 4597)
    of Sod, Couette and Poiseuille solves, served by the continuous-batching
    server within a 200 GB budget; requests arriving in [warm, duration) are
    measured.  Then the plain per-solve loop serves the same arrivals.  A
    spread of `sample` requests is re-run alone and compared bitwise."""
    import numpy as np
    import torch
    from paper_1905_04597_amd import serving
    from paper_1905_04597_amd import workloads as wl

    # start from an empty allocator cache: blocks cached by earlier phases of
    # other sizes would make the server's allocations free and re-allocate
    # device memory (a device-wide synchronisation) while it runs
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    arrivals = wl.served_requests(duration=duration)
    ids = set(int(i) for i in np.linspace(0, len(arrivals) - 1, sample))
    srv = serving.Server(keep_results=ids)
    t0 = time.perf_counter()
    reqs = srv.run(arrivals, max_seconds=duration + 60)
    served_wall = time.perf_counter() - t0
    summ = serving.summarize(reqs, (warm, duration))
    torch.cuda.synchronize()
    equal = all(_same_moments(r.result, serving.solve_alone(r.workload, r.steps)) for r in reqs if r.rid in ids)
    for r in reqs:
        r.result = None
    loop = serving.serve_per_solve(arrivals, max_seconds=loop_max)
    lsum = serving.summarize(loop, (warm, duration))
    eb = serving.ELEM_BYTES
    offered = sum(serving.step_bytes(w) * w.steps for _, w in arrivals) / duration
    return {
        "workload": "Poisson arrivals 200/s for %.0f s (first %.0f s warm-up), Sod (500..20000 nodes, 1000 steps) / "
                    "Couette / Poiseuille (Ny 32..2048, Nx 4..2048, 200 steps), level 1..7, log10 Kn U[-3,1], "
                    "FP32 or BF16 deviation storage, budget 200 GB, seeds 1905/4597" % (duration, warm),
        "offered_GBs": round(offered / 1e9, 1),
        "server": dict(summ, wall_s=round(served_wall, 2), peak_population_GB=round(srv.peak_in_use / 1e9, 2),
                       chunks=[l.chunks for l in srv.lanes]),
        "per_solve_loop": lsum,
        "alone_vs_mix_bitwise": equal, "alone_vs_mix_sample": len(ids),
    }


def run_served_rates(rates=(400.0, 800.0), duration: float = 6.0, warm: float = 1.0, loop_max: float = 45.0):
    """The served mix at higher arrival rates (same seeds and parameter
    distributions), server and per-solve loop: the sustained solves/s of
    each once the offered load exceeds what the loop can serve."""
    import torch
    from paper_1905_04597_amd import serving
    from paper_1905_04597_amd import workloads as wl

    out = []
    for rate in rates:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        arrivals = wl.served_requests(rate=rate, duration=duration)
        srv = serving.Server()
        reqs = srv.run(arrivals, max_seconds=duration + 60)
        summ = serving.summarize(reqs, (warm, duration))
        loop = serving.serve_per_solve(arrivals, max_seconds=loop_max)
        lsum = serving.summarize(loop, (warm, duration))
        offered = sum(serving.step_bytes(w) * w.steps for _, w in arrivals) / duration
        out.append({"rate_per_s": rate, "requests": len(arrivals), "offered_GBs": round(offered / 1e9, 1),
                    "server": {k: summ[k] for k in ("completed", "solves_per_s", "latency_p50_s", "latency_p99_s",
                                                    "failed")},
                    "per_solve_loop": {k: lsum[k] for k in ("completed", "solves_per_s", "latency_p50_s",
                                                            "latency_p99_s")}})
    return out


def _oracle_sample(args):
    """One oracle run of the bounded sample (a worker of cpu_baseline)."""
    level, nx, ny, steps = args
    import oracle

    s = oracle.OracleSolver(2, level, level, nx, ny, kn=0.1, bc_y=oracle.BC_WALL, g=1e-5)
    s.init_fields()
    s.step(1)
    t0 = time.perf_counter()
    s.step(steps)
    return time.perf_counter() - t0


def cpu_baseline(level: int = 5, nx: int = 64, ny: int = 1024, steps: int = 100, all_steps: int = 20):
    """The FP64 oracle (single-threaded C, as it stands) on a bounded sample
    of the workload: the same level, wall distance and parameters, a
    narrower channel.  One core: one run of `steps` steps.  All cores: one
    independent run of the same sample per core (processes), `all_steps`
    steps each, the aggregate node updates over the slowest run's time."""
    import multiprocessing as mp

    dt = _oracle_sample((level, nx, ny, steps))
    one = nx * ny * steps / dt / 1e9
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    # the host's share for this GPU (OMP_NUM_THREADS is set to it where the
    # cores are shared), at most 16 processes
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    cores = max(1, min(cores, share if share > 0 else cores, 16))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        times = pool.map(_oracle_sample, [(level, nx, ny, all_steps)] * cores)
    wall = time.perf_counter() - t0
    allc = cores * nx * ny * all_steps / max(times) / 1e9
    return {"value": one, "unit": "GLUPS", "cores": 1, "kind": "oracle",
            "sample": "G-D2Q(11x11) Poiseuille %dx%d (same ny, walls, g, Kn), %d steps, %.1f s, "
                      "single-threaded FP64 C" % (nx, ny, steps, dt),
            "all_cores": {"value": allc, "unit": "GLUPS", "cores": cores,
                          "sample": "%d independent oracle processes on the same sample, %d steps each, "
                                    "slowest %.1f s (%.1f s with start-up)" % (cores, all_steps, max(times), wall)}}


def load_traffic(storage: str):
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = t.get(storage)
    if not rec or t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", default="f32_shifted", choices=sorted(ELEM_BYTES))
    ap.add_argument("--level", type=int, default=5)
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--ny", type=int, default=1024)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--sweep-steps", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-only", action="store_true", help="print only the batched sweep record")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--batch-loop-steps", type=int, default=2000)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-only", action="store_true", help="print only the served-mix record")
    ap.add_argument("--served-seconds", type=float, default=12.0)
    ap.add_argument("--no-served-rates", action="store_true", help="skip the served mix at 400 and 800 requests/s")
    ap.add_argument("--only-3d", action="store_true", help="print only the three-dimensional sweep lines")
    a = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the hot path is a single-GPU lattice update "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        return 2

    import torch

    torch.cuda.set_device(0)
    if a.served_only:
        served = run_served(a.served_seconds)
        if not a.no_served_rates:
            served["rates"] = run_served_rates()
        print(json.dumps(served), flush=True)
        print(json.dumps(run_solves()), flush=True)
        return 0
    if a.only_3d:
        for levels, ev, shape in SWEEP_3D:
            print(json.dumps(run_gpu3(levels, ev, *shape, a.storage, a.sweep_steps, 5)), flush=True)
        return 0
    if a.batched_only:
        print(json.dumps(run_batched(a.batch_count, a.batch_steps, loop_steps=a.batch_loop_steps)), flush=True)
        return 0
    copy = copy_probe(reps=10 if not a.copy_probe else 20)
    ceiling = bandwidth_ceiling(reps=10)
    main_run = run_gpu(a.level, a.nx, a.ny, a.storage, a.steps, a.warmup)
    sweep = None
    if not a.no_sweep:
        sweep = []
        for lv in range(1, 8):
            r = run_gpu(lv, a.nx, a.ny, a.storage, a.sweep_steps, 5)
            sweep.append({"lattice": "odd", "N": lv})
            sweep[-1].update({k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()
                              if k in ("k", "Q", "glups", "achieved_GBs", "ms_per_step")})
            sweep[-1]["frac"] = round(r["achieved_GBs"] / PEAK_HBM_GBS, 4)
        # the G-D1Q(2N+2) lattices: D1Q3 x G-D1Q(2N+2) channels and the
        # symmetric products
        for lattice, levels in (("mixed_even", range(1, 14)), ("even", range(1, 8))):
            for lv in levels:
                r = run_gpu(lv, a.nx, a.ny, a.storage, a.sweep_steps, 5, lattice)
                sweep.append({"lattice": lattice, "N": lv, "Q": r["Q"], "glups": round(r["glups"], 4),
                              "achieved_GBs": round(r["achieved_GBs"], 4), "ms_per_step": round(r["ms_per_step"], 4),
                              "frac": round(r["achieved_GBs"] / PEAK_HBM_GBS, 4)})
                if r["ny"] != a.ny:
                    sweep[-1]["ny"] = r["ny"]
        # three dimensions
        for levels, ev, shape in SWEEP_3D:
            sweep.append(run_gpu3(levels, ev, *shape, a.storage, a.sweep_steps, 5))
        # the 16-bit storages over the 2N+1 levels (same lattice and size)
        for st in ("bf16_shifted_sr",):
            if st == a.storage:
                continue
            for lv in range(1, 8):
                r = run_gpu(lv, a.nx, a.ny, st, a.sweep_steps, 5)
                sweep.append({"lattice": "odd", "N": lv, "storage": st, "Q": r["Q"], "glups": round(r["glups"], 4),
                              "achieved_GBs": round(r["achieved_GBs"], 4), "ms_per_step": round(r["ms_per_step"], 4),
                              "frac": round(r["achieved_GBs"] / PEAK_HBM_GBS, 4)})
    batched = None if a.no_batched else run_batched(a.batch_count, a.batch_steps, loop_steps=a.batch_loop_steps)
    served = None if a.no_served else run_served(a.served_seconds)
    if served is not None and not a.no_served_rates:
        served["rates"] = run_served_rates()
    solves = None if a.no_served else run_solves()
    cpu = None if a.no_cpu_baseline else cpu_baseline(a.level)
    achieved = main_run["achieved_GBs"]
    line = {
        "metric": "GLUPS (Poiseuille G-D2Q(11x11) 4096x1024 stream-collide) and % HBM roofline",
        "value": round(main_run["glups"], 4),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[a.storage],
        "data": "synthetic",
        "config": {
            "workload": "force-driven Poiseuille, G-D2Q(%dx%d) (k=%d), %dx%d nodes, diffuse walls, "
                        "g=1e-5, Kn=0.1, from rest" % (2 * a.level + 1, 2 * a.level + 1, a.level - 1, a.nx, a.ny),
            "storage": a.storage,
            "nodes": a.nx * a.ny,
            "velocities": main_run["Q"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": load_traffic(a.storage),
            "bytes_per_launch": main_run["bytes_per_launch"],
            "copy_kernel_GBs": ceiling["copy_GBs"],
            "frac_of_copy_kernel": round(achieved / ceiling["copy_GBs"], 4),
            "streaming_kernels": ceiling,
            "torch_copy_GBs": copy["GBs"],
        },
        "cpu_baseline": cpu,
        "mass_drift_rel": main_run["mass_drift_rel"],
    }
    if sweep is not None:
        line["per_k"] = sweep
    if batched is not None:
        line["batched_sweep"] = batched
    if served is not None:
        line["served_mix"] = served
    if solves is not None:
        line["single_solves"] = solves
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
