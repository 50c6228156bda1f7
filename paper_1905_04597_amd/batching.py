"""Batched stepping of many channel instances: schedule autotuner.

A :class:`~paper_1905_04597_amd.glbm.Batch` advances its members with one
launch per kernel variant and step over a table of tiles (a tile is a run of
nodes of one member), optionally replayed from a captured HIP graph.  Five
choices shape the schedule:

* ``tile_nodes`` - nodes per workgroup (64, 128 or 256).  Small tiles waste
  fewer lanes on the ragged ends of small members; large tiles have more
  waves per workgroup to hide memory latency.
* ``order`` - how members' tiles are laid out along the grid: contiguous per
  member, dealt round-robin over members (spreads each member's rows over
  the accelerator's dies), or contiguous by decreasing work.
* ``graph_steps`` - steps per captured graph (0 = plain launches): graphs
  remove the host cost of one launch per variant and step.
* ``resident_nodes`` - members up to this size are stepped by one workgroup
  each, every step of a chunk in one launch (a per-instance schedule: small
  lattices leave the per-step launches).
* ``streams`` - kernel variants advance side by side on up to this many
  streams (1, 4 or 8; at most one per variant), so that the tail of one
  variant's launch overlaps the others.

:func:`autotune` times every candidate on scratch copies of the members
(fresh lattices of the same configurations, initialised at rest) and
returns the fastest, so tuning never disturbs the real members.
"""
from __future__ import annotations

import itertools
import time

from . import glbm

TILE_NODES = (64, 128, 256)
ORDERS = ("member", "interleave", "largest_first")
GRAPH_STEPS = (0, 32)
RESIDENT_NODES = (0, 8192)
STREAMS = (1, 4, 8)


def candidates(tiles=TILE_NODES, orders=ORDERS, graphs=GRAPH_STEPS, resident=RESIDENT_NODES, streams=STREAMS):
    return [dict(tile_nodes=t, order=o, graph_steps=g, resident_nodes=r, streams=n)
            for t, o, g, r, n in itertools.product(tiles, orders, graphs, resident, streams)]


def time_batch(solvers, options: dict, steps: int, warmup: int = 2) -> float:
    """Seconds per step of a batch of `solvers` under `options` (GPU events on
    the batch's stream)."""
    import torch

    with glbm.Batch(solvers, **options) as b:
        b.step(max(warmup, options.get("graph_steps", 0)))
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record()
        b.step(steps)
        stop.record()
        torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3 / steps


def autotune(configs, steps: int = 64, cands=None, memory_cap: int = 64 << 30, verbose: bool = False):
    """Pick the fastest schedule for a batch of these configurations.

    configs: glbm.Config objects (or workloads).  Builds scratch solvers of
    the same shapes (refuses if their population buffers would exceed
    `memory_cap` bytes), times each candidate for `steps` steps (a multiple
    of every candidate's graph length keeps the comparison fair) and
    returns (best options, [(options, seconds per step), ...])."""
    cfgs = [c if isinstance(c, glbm.Config) else glbm.config_from_workload(c) for c in configs]
    need = sum(2 * glbm.population_bytes(c) for c in cfgs)
    if need > memory_cap:
        raise glbm.GlbmError("autotune needs %d bytes of scratch lattices, above the cap %d" % (need, memory_cap))
    cands = cands or candidates()
    scratch = [glbm.Solver(c) for c in cfgs]
    results = []
    try:
        for s in scratch:
            s.init_fields()
        for opt in cands:
            t0 = time.perf_counter()
            sec = time_batch(scratch, opt, steps)
            results.append((opt, sec))
            if verbose:
                print("[autotune] %s: %.1f us/step (%.2f s)" % (opt, sec * 1e6, time.perf_counter() - t0), flush=True)
    finally:
        for s in scratch:
            s.close()
    best = min(results, key=lambda r: r[1])[0]
    return best, results
