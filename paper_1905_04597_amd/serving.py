"""Continuous-batching server for lattice solves on one GPU.

Requests (a lattice configuration and a step budget) arrive over time.  The
server keeps every admitted request's populations resident in device memory
and advances all of them together, a chunk of steps at a time, through
batches (glbm_batch_*: one launch per kernel variant and step over a table of
tiles).  Between chunks, finished requests leave (their moments are computed
on the device and the populations released) and waiting requests join, as
slots and the device-memory budget allow: continuous batching, not a queue.

Requests are split over lanes, each a batch on its own stream: one lane for
the large solves and several for the small ones (most requests, little
traffic), so that the small solves are not held to the pace of the large
ones.  The small solves are spread over their lanes by kernel variant, so the
lanes' launches proceed side by side on the GPU's hardware queues, and the
smallest of them run resident (one workgroup, a whole chunk of steps per
launch).  A lane re-plans its batch in place (glbm_batch_update) when its
members change.

Admission: the device bytes of all active requests (glbm_required_bytes
each: both population buffers and the statistics buffers) stay within the
budget (default 200 GB); requests
are admitted first come, first served per lane (a request that does not fit
waits, and so do the ones behind it in its lane).

Every request's result is bitwise the result of the same solve run alone,
because a batched lattice runs exactly the single-lattice kernel code.

Failure detection: when a request finishes, the server reads its FP64
diagnostics (glbm_stats_static, which allocates nothing: the server's calls
come from one thread and each one synchronises, so they never overlap) and
records its health: "ok", "positivity" (some
node left the domain where the equilibrium is non-negative, section 3: the
result is kept, flagged) or "nonfinite" (the solve blew up: the request is
retired as failed, with no result).  With check_every > 0 the members of a
lane are also checked every that many chunks, and a blown-up request is
retired at once instead of running out its step budget.
"""
from __future__ import annotations

import collections
import dataclasses
import time
import zlib
from typing import Optional

import numpy as np

from . import glbm
from . import workloads as wl

ELEM_BYTES = {"f32": 4, "f32_shifted": 4, "bf16_shifted": 2, "bf16_shifted_sr": 2}


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    workload: wl.Workload
    steps: int
    # filled in by the server
    lane: int = -1
    nbytes: int = 0           # device bytes of the two population buffers
    admitted: Optional[float] = None
    finished: Optional[float] = None
    result: Optional[dict] = None   # device moments {rho, ux, uy, T, pxy} when kept
    health: Optional[str] = None    # "ok", "positivity" or "nonfinite" (then failed, no result)
    f0: Optional[np.ndarray] = None  # initial populations [Q][ny][nx] instead of the workload's init

    @property
    def failed(self) -> bool:
        return self.health == "nonfinite"

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


def step_bytes(w: wl.Workload) -> int:
    """Algorithmic HBM bytes of one step (read + write every population)."""
    return 2 * w.nodes * w.nvel * ELEM_BYTES[w.storage]


def lane_of(w: wl.Workload, light_bytes: int, light_lanes: int) -> int:
    """Lane of a request: the heavy lane (index light_lanes) when one step
    moves at least light_bytes, else a light lane chosen by the kernel
    variant (axes, storage, boundaries), so that the members of one variant
    share a lane and its launches."""
    if step_bytes(w) >= light_bytes:
        return light_lanes
    key = "%d/%d%s/%d%s/%s/%s/%s" % (w.dims, w.level_x, "e" if w.even_x else "", w.level_y,
                                      "e" if w.even_y else "", w.storage, w.bc_x, w.bc_y)
    return zlib.crc32(key.encode()) % light_lanes


def admissible(waiting_bytes, in_use: float, budget: float, free_slots: int) -> int:
    """How many requests at the head of a lane's queue to admit now, first
    come first served: each needs its population bytes within the budget
    beside those in use and a free slot; the first that does not fit stops
    the admission (no overtaking)."""
    n = 0
    for nb in waiting_bytes:
        if n >= free_slots or in_use + nb > budget:
            break
        in_use += nb
        n += 1
    return n


def make_solver(w: wl.Workload, stream, f0=None):
    """Create and initialise the solver of a request on `stream` (its buffers
    are allocated from that stream, so their reuse is ordered on it); f0, if
    given, are its initial populations."""
    import torch

    with torch.cuda.stream(stream):
        s = glbm.solver_for(w, stream=stream)
        if f0 is not None:
            s.init_populations(f0)
        elif w.init == "sod":
            rho = wl.sod_density(w.nx, w.end_rho[0], w.end_rho[1])
            s.init_fields(rho, np.zeros_like(rho))
        else:
            s.init_fields()
    return s


def solve_alone(w: wl.Workload, steps: int, stream=None, f0=None) -> dict:
    """The same solve without the server: one lattice, one launch per step."""
    import torch

    stream = stream or torch.cuda.current_stream()
    s = make_solver(w, stream, f0)
    s.step(steps)
    with torch.cuda.stream(stream):
        m = s.moments()
    stream.synchronize()
    s.close()
    return m


class _Active:
    __slots__ = ("req", "solver", "left")

    def __init__(self, req, solver, left):
        self.req, self.solver, self.left = req, solver, left


class _Lane:
    def __init__(self, index, chunk, slots, batch_opts):
        import torch

        self.index = index
        self.chunk = chunk
        self.slots = slots
        self.batch_opts = batch_opts
        self.stream = torch.cuda.Stream()
        self.event = torch.cuda.Event()
        self.busy = False
        self.batch = None
        self.members: list = []
        self.leaving: list = []
        self.changed = False
        self.waiting = collections.deque()
        self.chunks = 0


class Server:
    """Continuous batching over light lanes (small requests, by kernel
    variant) and one heavy lane (large requests).

    hbm_budget: bytes of population buffers the active requests may hold.
    light_bytes: a request whose step moves fewer bytes goes to a light lane.
    light_lanes: number of light lanes.
    chunks: steps per chunk in a (light, heavy) lane.
    slots: most active requests per (light, heavy) lane.
    resident_nodes: light-lane members of at most this many nodes run
    resident (glbm_batch_options.resident_nodes).
    streams: streams per lane over which a lane's kernel variants advance side
    by side (glbm_batch_options.streams); (light, heavy).
    keep_results: True, or a set of request ids, whose device moments
    {rho, ux, uy, T, pxy} are kept in Request.result.
    check_every: also check the health of every member of a lane every that
    many of its chunks (0: only when a request finishes)."""

    def __init__(self, hbm_budget: float = 200e9, light_bytes: int = 64 << 20, light_lanes: int = 3,
                 chunks=(50, 20), slots=(4096, 256), tile_nodes: int = 128, order: str = "interleave",
                 resident_nodes: int = 2048, streams=(1, 1), keep_results: bool = False,
                 check_every: int = 0, clock=time.perf_counter):
        self.check_every = int(check_every)
        self.hbm_budget = float(hbm_budget)
        self.light_bytes = int(light_bytes)
        self.keep_results = keep_results
        self.clock = clock
        light = dict(tile_nodes=tile_nodes, order=order, graph_steps=0, resident_nodes=resident_nodes,
                     streams=int(streams[0]))
        heavy = dict(tile_nodes=tile_nodes, order=order, graph_steps=0, resident_nodes=0, streams=int(streams[1]))
        self.nlight = int(light_lanes)
        self.lanes = [_Lane(i, chunks[0], slots[0], light) for i in range(self.nlight)]
        self.lanes.append(_Lane(self.nlight, chunks[1], slots[1], heavy))
        self.in_use = 0
        self.peak_in_use = 0

    def _lane_of(self, w) -> int:
        return lane_of(w, self.light_bytes, self.nlight)

    def _keep(self, req) -> bool:
        k = self.keep_results
        return bool(k) if isinstance(k, bool) else req.rid in k

    # ---------------------------------------------------------------- lanes
    def _retire(self, lane: _Lane, now: float):
        """Finished members: record the time and compute their moments (a
        member of a batch may be observed); they leave at the next plan."""
        import torch

        if self.check_every > 0 and lane.chunks and lane.chunks % self.check_every == 0:
            for a in lane.members:
                if a.left > 0 and a.solver.stats(static=True)["health"] == "nonfinite":
                    a.left = 0  # blown up: retire it now
        done = [a for a in lane.members if a.left <= 0]
        if not done:
            return
        lane.members = [a for a in lane.members if a.left > 0]
        lane.changed = True
        for a in done:
            a.req.finished = now
            # the lane's work is done (its event was reached): this reads the
            # finished state at once
            a.req.health = a.solver.stats(static=True)["health"]
            if self._keep(a.req) and not a.req.failed:
                with torch.cuda.stream(lane.stream):
                    a.req.result = a.solver.moments()
            lane.leaving.append(a)

    def _admit(self, lane: _Lane, now: float):
        n = admissible((r.nbytes for r in lane.waiting), self.in_use, self.hbm_budget,
                       lane.slots - len(lane.members))
        for _ in range(n):
            r = lane.waiting.popleft()
            s = make_solver(r.workload, lane.stream, r.f0)
            r.admitted = now
            self.in_use += r.nbytes
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            lane.members.append(_Active(r, s, r.steps))
            lane.changed = True

    def _launch(self, lane: _Lane):
        sol = [a.solver for a in lane.members]
        if lane.batch is None:
            if sol:
                lane.batch = glbm.Batch(sol, stream=lane.stream, **lane.batch_opts)
        elif lane.changed:
            lane.batch.update(sol)
        lane.changed = False
        # the finished solvers are out of the batch now: release them (their
        # buffers return to the lane stream's pool after the work queued on it)
        for a in lane.leaving:
            a.solver.close()
            a.solver = None
            self.in_use -= a.req.nbytes
        lane.leaving = []
        if not lane.members:
            lane.busy = False
            return
        k = min(lane.chunk, min(a.left for a in lane.members))
        lane.batch.step(k)
        for a in lane.members:
            a.left -= k
        lane.event.record(lane.stream)
        lane.busy = True
        lane.chunks += 1

    # ------------------------------------------------------------------ run
    def run(self, arrivals, max_seconds: float = 120.0):
        """Serve [(arrival seconds, Workload)] (or (arrival, Workload, f0)
        with initial populations f0) in real time; returns the Request records
        (every request finished unless max_seconds ran out)."""
        reqs = [Request(i, a[0], a[1], a[1].steps, f0=a[2] if len(a) > 2 else None) for i, a in enumerate(arrivals)]
        for r in reqs:
            r.nbytes = glbm.required_bytes(glbm.config_from_workload(r.workload))
            if r.nbytes > self.hbm_budget:
                raise glbm.GlbmError("request %d needs %d bytes, above the budget" % (r.rid, r.nbytes))
            r.lane = self._lane_of(r.workload)
        pending = collections.deque(sorted(reqs, key=lambda r: r.arrival))
        t0 = self.clock()
        while True:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                self.lanes[r.lane].waiting.append(r)
            for lane in self.lanes:
                if lane.busy and not lane.event.query():
                    continue
                now = self.clock() - t0
                self._retire(lane, now)
                self._admit(lane, now)
                self._launch(lane)
            idle = not any(l.busy for l in self.lanes)
            if idle and not pending and not any(l.waiting for l in self.lanes):
                break
            if now > max_seconds:
                break
            if idle and pending:
                # nothing on the GPU: wait for the next arrival
                time.sleep(max(0.0, min(1e-3, pending[0].arrival - (self.clock() - t0))))
        self.close()
        return reqs

    def close(self):
        for lane in self.lanes:
            lane.stream.synchronize()
            if lane.batch is not None:
                lane.batch.update([])
                lane.batch.close()
                lane.batch = None
            for a in lane.members + lane.leaving:
                a.solver.close()
                self.in_use -= a.req.nbytes
            lane.members = []
            lane.leaving = []


def serve_per_solve(arrivals, max_seconds: float = 120.0, clock=time.perf_counter):
    """The plain per-solve loop on the same arrivals: each request alone, in
    arrival order, one launch per step, its moments computed before the next
    one starts."""
    import torch

    reqs = [Request(i, t, w, w.steps) for i, (t, w) in enumerate(arrivals)]
    stream = torch.cuda.current_stream()
    t0 = clock()
    for r in sorted(reqs, key=lambda r: r.arrival):
        now = clock() - t0
        if now > max_seconds:
            break
        if r.arrival > now:
            time.sleep(r.arrival - now)
        r.admitted = clock() - t0
        s = make_solver(r.workload, stream)
        s.step(r.steps)
        s.moments()
        stream.synchronize()
        s.close()
        r.finished = clock() - t0
    return reqs


def summarize(reqs, window=(2.0, 12.0)) -> dict:
    """Throughput and latency of the requests that arrived inside `window`."""
    lo, hi = window
    meas = [r for r in reqs if lo <= r.arrival < hi]
    done = [r for r in meas if r.finished is not None]
    lat = np.array(sorted(r.latency for r in done)) if done else np.array([np.nan])
    span = (max(r.finished for r in done) - lo) if done else float("nan")
    return {
        "requests": len(meas), "completed": len(done),
        "solves_per_s": round(len(done) / span, 2) if done else 0.0,
        "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
        "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
        "latency_max_s": round(float(lat.max()), 4),
        "node_steps": int(sum(r.workload.nodes * r.steps for r in done)),
        "failed": sum(1 for r in done if r.failed),
        "positivity_flagged": sum(1 for r in done if r.health == "positivity"),
    }
