"""Summaries of rocprofv3 output for the step kernel (kernel trace and memory
counters), written as short text under ``profiles/``.

    python -m paper_1905_04597_amd.profiling --workload NAME --storage S \\
        --trace DIR/kt_results.db --fetch DIR/pmc_results.db --write DIR/pmc_results.db \\
        --command "the rocprofv3 command lines" [--copy-bytes 2147483648]
    python -m paper_1905_04597_amd.profiling batched --trace DIR/kt_results.db --command "..."

The memory counters FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled
by what they read for a plain device copy of known size in the same run
(bench.py copies 2 GiB before timing), giving HBM bytes per launch of the
step kernel; the result is recorded, with a hash of the kernel sources, in
``profiles/traffic_<workload>.json`` for bench.py to report.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")
# kernels of known byte count for scaling the memory counters: the library's
# own copy kernel (glbm_bandwidth_probe, bench.py runs it on 2 GiB), else the
# HIP runtime's device copy
COPY_KERNELS = ("probe_copy", "__amd_rocclr_copyBuffer")
SOURCES = ("glbm_device.h", "glbm_device3.h", "glbm_inst.hip", "glbm_inst3.hip", "glbm_api.hip")


def kernel_source_hash() -> str:
    """Hash of the kernel sources: recorded traffic is used only while it
    matches."""
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(ROOT, "paper_1905_04597_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_stats(db_path: str):
    db = sqlite3.connect(db_path)
    rows = list(db.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    # top_kernels reports microseconds
    return [dict(name=r[0], calls=int(r[1]), total_us=float(r[2]), avg_us=float(r[3]), pct=float(r[4]))
            for r in rows]


def counter(db_path: str, name: str):
    """Median value (KiB) per kernel name and grid size."""
    db = sqlite3.connect(db_path)
    by = {}
    for k, v, g in db.execute("select kernel_name, value, grid_size from counters_collection where counter_name=?",
                              (name,)):
        by.setdefault((k, int(g)), []).append(float(v))
    return {key: statistics.median(vs) for key, vs in by.items()}


def batched_busy(trace: str):
    """Microseconds during which at least one batched step kernel ran (the
    union of their dispatch intervals), and the number of steps (launches of
    the most launched level)."""
    db = sqlite3.connect(trace)
    iv = sorted((int(a), int(b)) for a, b in db.execute(
        "select start, end from kernels where name like '%batch_step_kernel%'"))
    calls = {}
    for (name,) in db.execute("select name from kernels where name like '%batch_step_kernel%'"):
        calls[name] = calls.get(name, 0) + 1
    busy, cur_a, cur_b = 0, None, None
    for a, b in iv:
        if cur_b is None or a > cur_b:
            if cur_b is not None:
                busy += cur_b - cur_a
            cur_a, cur_b = a, b
        else:
            cur_b = max(cur_b, b)
    if cur_b is not None:
        busy += cur_b - cur_a
    steps = max(calls.values()) if calls else 0
    return busy / 1e3, steps


def batched_summary(trace: str, command: str, count: int = 512, storage: str = "f32_shifted"):
    """Per-level averages of the batched step kernel over the channel sweep:
    each launch steps every instance of one level once, so its algorithmic
    bytes are the sum of 2 Q s nodes over those instances."""
    import re

    from . import workloads as wl

    eb = 4 if storage.startswith("f32") else 2
    per_level = {}
    for w in wl.sweep_workloads(count, storage=storage):
        per_level[w.level_x] = per_level.get(w.level_x, 0) + 2 * w.nvel * eb * w.nodes
    stats = kernel_stats(trace)
    rows = []
    for st in stats:
        m = re.search(r"batch_step_kernel<(\d+), (\d+), (\d+), (\d+), (\d+), (\d+)>", st["name"])
        if not m:
            continue
        lx = int(m.group(1))
        b = per_level.get(lx)
        if b is None:
            continue
        rows.append((lx, st["calls"], st["avg_us"], b, b / (st["avg_us"] * 1e-6) / 1e9))
    rows.sort()
    path = os.path.join(PROFILES, "batch_step_kernel_channel_sweep_%d.md" % count)
    with open(path, "w") as fh:
        fh.write("# Batched step kernel, channel sweep of %d instances (Nx = 4, storage %s)\n\n" % (count, storage))
        fh.write("Command (run on one MI355X):\n\n```\n%s\n```\n\n" % command.strip())
        fh.write("## rocprofv3 --kernel-trace --stats (top kernels)\n\n| kernel | calls | avg us | total us | % |\n"
                 "|---|---|---|---|---|\n")
        for st in stats[:12]:
            fh.write("| `%s` | %d | %.1f | %.1f | %.2f |\n" % (st["name"][:90], st["calls"], st["avg_us"], st["total_us"],
                                                           st["pct"]))
        fh.write("\n## Per level: one launch steps every instance of the level once\n\n"
                 "| level N | launches | avg us | algorithmic bytes / launch | GB/s |\n|---|---|---|---|---|\n")
        for lx, calls, avg, b, gbs in rows:
            fh.write("| %d | %d | %.1f | %.4g | %.0f |\n" % (lx, calls, avg, b, gbs))
        tot_us = sum(r[2] for r in rows)
        tot_b = sum(r[3] for r in rows)
        busy_us, steps = batched_busy(trace)
        fh.write("\nSum of the per-level launch times: %.1f us per step (launches of different levels overlap "
                 "when the batch runs its variants on several streams, each then taking longer).\n" % tot_us)
        if steps:
            fh.write("\nOne step of the whole sweep: %.1f us with batched kernels running (union of their "
                     "intervals over the %d batched steps of the run, the autotuner's trials of every schedule "
                     "included) for %.4g algorithmic bytes, %.0f GB/s.\n"
                     % (busy_us / steps, steps, tot_b, tot_b / (busy_us / steps * 1e-6) / 1e9))
        fh.write("- kernel source hash: %s\n" % kernel_source_hash())
    print(path)


def three_d_summary(trace: str, command: str, steps: int = 20, storage: str = "f32_shifted"):
    """Kernel trace of the three-dimensional lattices of the bench sweep:
    average duration of each lattice's step kernel, and the algorithmic HBM
    rate 2 Q s nodes / duration."""
    import re

    eb = 4 if storage.startswith("f32") else 2
    # axis codes: N for G-D1Q(2N+1), 16 + N for G-D1Q(2N+2)
    shapes = {(1, 1, 1): (27, 256 * 256 * 128), (2, 2, 2): (125, 128 ** 3), (3, 3, 3): (343, 128 ** 3)}
    for n in range(2, 8):
        shapes[(1, n, 1)] = (9 * (2 * n + 1), 256 * 128 * 128)
        shapes[(1, 16 + n, 1)] = (9 * (2 * n + 2), 256 * 128 * 128)
    stats = kernel_stats(trace)
    path = os.path.join(PROFILES, "step3_kernel_3d_sweep_%s.md" % storage)
    with open(path, "w") as fh:
        fh.write("# Three-dimensional step kernels, bench sweep shapes (storage %s)\n\n" % storage)
        fh.write("Command (run on one MI355X):\n\n```\n%s\n```\n\n" % command.strip())
        fh.write("## rocprofv3 --kernel-trace --stats (top kernels)\n\n| kernel | calls | avg us | total us | % |\n"
                 "|---|---|---|---|---|\n")
        for st in stats[:12]:
            fh.write("| `%s` | %d | %.1f | %.1f | %.2f |\n" % (st["name"][:90], st["calls"], st["avg_us"], st["total_us"],
                                                           st["pct"]))
        # a step with walls is the wall pre-pass (the per-column wall
        # factors) and the step kernel: both count
        pre = {}
        for st in stats:
            m = re.search(r"wall_rate3_kernel<(\d+), (\d+), (\d+),", st["name"])
            if m:
                pre[tuple(int(g) for g in m.groups())] = st["avg_us"]
        fh.write("\n## Steps\n\n| lattice (axis codes x, y, z) | Q | nodes | step kernel avg us | wall pre-pass avg us |"
                 " algorithmic GB/s of the step |\n|---|---|---|---|---|---|\n")
        for st in stats:
            m = re.search(r"step3_(?:split_)?kernel<(\d+), (\d+), (\d+),", st["name"])
            if not m:
                continue
            key = tuple(int(g) for g in m.groups())
            if key not in shapes:
                continue
            q, nodes = shapes[key]
            us = st["avg_us"] + pre.get(key, 0.0)
            fh.write("| %s | %d | %d | %.1f | %.1f | %.0f |\n" % (key, q, nodes, st["avg_us"], pre.get(key, 0.0),
                                                               2 * q * eb * nodes / (us * 1e-6) / 1e9))
    print(path)


def _csv_rows(path: str):
    import csv

    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def counters_summary(workload: str, tag: str, trace_csv: str, pmc_csvs, command: str, match: str = "glbm::step",
                     compiler=None):
    """Per-kernel medians of the SQ/TCC counters of the step kernel(s) and the
    calibration copy kernel, with the register counts of the kernel trace,
    written to profiles/counters_<workload>_<tag>.md.

    Units: instruction counters are per wave (summed over waves); SQ_WAVE_CYCLES,
    SQ_WAIT_INST_ANY and SQ_ACTIVE_INST_* count 4-cycle units summed over waves;
    SQ_BUSY_CU_CYCLES counts cycles summed over compute units; GRBM_GUI_ACTIVE
    counts cycles summed over the 8 XCDs.  Hence mean resident waves per CU =
    4 SQ_WAVE_CYCLES / SQ_BUSY_CU_CYCLES, the fraction of wave time waiting =
    SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES, and VALU busy per SIMD =
    SQ_ACTIVE_INST_VALU / SQ_BUSY_CU_CYCLES (4 SIMDs per CU, 4 cycles per
    wave64 instruction)."""
    vals = {}
    for path in pmc_csvs:
        for r in _csv_rows(path):
            k = r["Kernel_Name"]
            if match in k or "probe_copy" in k:
                vals.setdefault((k, int(r["Grid_Size"])), {}).setdefault(r["Counter_Name"], []).append(
                    float(r["Counter_Value"]))
    durs = {}
    for r in _csv_rows(trace_csv):
        k = r["Kernel_Name"]
        if match in k or "probe_copy" in k:
            durs.setdefault((k, int(r["Grid_Size_X"])), []).append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    md = os.path.join(PROFILES, "counters_%s_%s.md" % (workload, tag))
    with open(md, "w") as fh:
        fh.write("# Counters of the step kernel, %s, %s\n\n" % (workload, tag))
        fh.write("Commands (run on one MI355X):\n\n```\n%s\n```\n\n" % command.strip())
        fh.write("Medians per dispatch.  Mean resident waves per CU = 4 SQ_WAVE_CYCLES / SQ_BUSY_CU_CYCLES "
                 "(8 = two waves per SIMD); waiting = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES; VALU busy per SIMD = "
                 "SQ_ACTIVE_INST_VALU / SQ_BUSY_CU_CYCLES; L2 hit rate = TCC_HIT / (TCC_HIT + TCC_MISS).  The "
                 "library's copy kernel (2 GiB each way) is the reference.\n\n")
        fh.write("| kernel | grid | trace median us | waves | VALU insts per wave | "
                 "VMEM rd / wr per wave | waves per CU | waiting | VALU busy | L2 hit |\n")
        fh.write("|---|---|---|---|---|---|---|---|---|---|\n")
        for (k, g), c in sorted(vals.items(), key=lambda kv: (("probe" in kv[0][0]), kv[0][1])):
            m = {n: statistics.median(v) for n, v in c.items()}
            w = m.get("SQ_WAVES", float("nan"))
            busy = m.get("SQ_BUSY_CU_CYCLES", float("nan"))
            wc = m.get("SQ_WAVE_CYCLES", float("nan"))
            hit, miss = m.get("TCC_HIT_sum", float("nan")), m.get("TCC_MISS_sum", float("nan"))
            du = durs.get((k, g))
            short = "glbm_bandwidth_probe copy" if "probe_copy" in k else k.split("(")[0][:48]
            fh.write("| `%s` | %d | %s | %.0f | %.0f | %.0f / %.0f | %.2f | %.2f | %.2f | %.2f |\n" % (
                short, g,
                ("%.1f" % statistics.median(du)) if du else "-", w, m.get("SQ_INSTS_VALU", float("nan")) / w,
                m.get("SQ_INSTS_VMEM_RD", float("nan")) / w, m.get("SQ_INSTS_VMEM_WR", float("nan")) / w,
                4 * wc / busy, m.get("SQ_WAIT_INST_ANY", float("nan")) / wc,
                m.get("SQ_ACTIVE_INST_VALU", float("nan")) / busy, hit / (hit + miss)))
        if compiler:
            fh.write("\nRegisters per lane from the compiler's resource report (hipcc -O3 --offload-arch=gfx950 "
                     "-Rpass-analysis=kernel-resource-usage on the kernel sources): %s.\n" % compiler)
    print(md)
    return md


def main(argv=None):
    import sys

    argv = sys.argv[1:] if argv is None else argv
    if argv and argv[0] == "counters":
        cp = argparse.ArgumentParser()
        cp.add_argument("--workload", required=True)
        cp.add_argument("--tag", required=True)
        cp.add_argument("--trace-csv", required=True)
        cp.add_argument("--pmc-csv", action="append", required=True)
        cp.add_argument("--command", required=True)
        cp.add_argument("--compiler", default=None, help="register counts from the compiler's resource report")
        c = cp.parse_args(argv[1:])
        return counters_summary(c.workload, c.tag, c.trace_csv, c.pmc_csv, c.command, compiler=c.compiler)
    if argv and argv[0] == "three_d":
        tp = argparse.ArgumentParser()
        tp.add_argument("--trace", required=True)
        tp.add_argument("--command", required=True)
        tp.add_argument("--storage", default="f32_shifted")
        t = tp.parse_args(argv[1:])
        return three_d_summary(t.trace, t.command, storage=t.storage)
    if argv and argv[0] == "batched":
        bp = argparse.ArgumentParser()
        bp.add_argument("--trace", required=True)
        bp.add_argument("--command", required=True)
        bp.add_argument("--count", type=int, default=512)
        b = bp.parse_args(argv[1:])
        return batched_summary(b.trace, b.command, b.count)
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--storage", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--copy-bytes", type=int, default=2 << 30)
    ap.add_argument("--algorithmic-bytes", type=float, required=True)
    a = ap.parse_args(argv)

    stats = kernel_stats(a.trace)
    fetch = counter(a.fetch, "FETCH_SIZE")
    write = counter(a.write, "WRITE_SIZE")
    copy_key = None
    for name in COPY_KERNELS:
        keys = [k for k in fetch if name in k[0] and k in write]
        if keys:
            copy_key = max(keys, key=lambda k: fetch[k])
            break
    f_scale = a.copy_bytes / (fetch[copy_key] * 1024.0)
    w_scale = a.copy_bytes / (write[copy_key] * 1024.0)
    # a time step may be more than one launch (16-bit storage with walls:
    # interior rows and wall rows): sum the step kernels
    step_keys = [k for k in fetch if "glbm::step_kernel" in k[0]]
    step_stats = [s for s in stats if "glbm::step_kernel" in s["name"]]
    avg_us = sum(s["avg_us"] for s in step_stats)
    fkib = sum(fetch[k] for k in step_keys)
    wkib = sum(write.get(k, 0.0) for k in step_keys)
    fb = fkib * 1024.0 * f_scale
    wb = wkib * 1024.0 * w_scale
    rec = {
        "kernel": " + ".join(k[0] for k in step_keys), "grid": [k[1] for k in step_keys], "avg_duration_us": avg_us,
        "fetch_kib_raw": fkib, "write_kib_raw": wkib,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "hbm_fetch_bytes_per_launch": fb, "hbm_write_bytes_per_launch": wb,
        "hbm_bytes_per_launch": fb + wb, "algorithmic_bytes_per_launch": a.algorithmic_bytes,
        "traffic_over_algorithmic": (fb + wb) / a.algorithmic_bytes,
        "hbm_GBs": (fb + wb) / (avg_us * 1e-6) / 1e9,
    }
    os.makedirs(PROFILES, exist_ok=True)
    tpath = os.path.join(PROFILES, "traffic_%s.json" % a.workload)
    allrec = {}
    if os.path.exists(tpath):
        with open(tpath) as fh:
            allrec = json.load(fh)
    if allrec.get("kernel_source_hash") != kernel_source_hash():
        allrec = {}
    allrec["kernel_source_hash"] = kernel_source_hash()
    allrec[a.storage] = rec
    with open(tpath, "w") as fh:
        json.dump(allrec, fh, indent=1)

    md = os.path.join(PROFILES, "step_kernel_%s_%s.md" % (a.workload, a.storage))
    with open(md, "w") as fh:
        fh.write("# Step kernel, %s, storage %s\n\n" % (a.workload, a.storage))
        fh.write("Commands (run on one MI355X):\n\n```\n%s\n```\n\n" % a.command.strip())
        fh.write("## rocprofv3 --kernel-trace --stats\n\n| kernel | calls | avg us | total us | % |\n|---|---|---|---|---|\n")
        for s in stats[:8]:
            fh.write("| `%s` | %d | %.1f | %.1f | %.2f |\n" % (s["name"][:70], s["calls"], s["avg_us"], s["total_us"], s["pct"]))
        fh.write("\n## Memory counters (median KiB per dispatch)\n\n| kernel | grid | FETCH_SIZE | WRITE_SIZE |\n|---|---|---|---|\n")
        for k in sorted(set(fetch) | set(write), key=lambda k: -fetch.get(k, 0)):
            if fetch.get(k, 0) + write.get(k, 0) < 1024:
                continue
            fh.write("| `%s` | %d | %.1f | %.1f |\n" % (k[0][:60], k[1], fetch.get(k, float("nan")), write.get(k, float("nan"))))
        fh.write("\nCalibration: the %d-byte device copy (`%s`) reads FETCH_SIZE x %.3f and WRITE_SIZE x %.3f "
                 "of its true bytes.\n\n" % (a.copy_bytes, copy_key[0][:60], 1 / f_scale, 1 / w_scale))
        fh.write("## Step kernel(s) per time step\n\n")
        fh.write("- average duration: %.1f us\n" % rec["avg_duration_us"])
        fh.write("- HBM bytes (scaled counters): fetch %.4g, write %.4g, total %.4g\n" % (fb, wb, fb + wb))
        fh.write("- algorithmic bytes 2 Q s per node: %.4g (traffic / algorithmic = %.3f)\n"
                 % (a.algorithmic_bytes, rec["traffic_over_algorithmic"]))
        fh.write("- HBM rate from the counters: %.0f GB/s\n" % rec["hbm_GBs"])
        fh.write("- kernel source hash: %s\n" % kernel_source_hash())
    print(md)
    print(tpath)


if __name__ == "__main__":
    main()
