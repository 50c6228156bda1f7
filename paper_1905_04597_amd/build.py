"""Build libglbm.so for gfx950 with hipcc (in-tree).

Usage: python -m paper_1905_04597_amd.build [--jobs J] [--incremental]

Every (axis kind, row layout, hierarchy level) is compiled as its own object
(they are the slow part), in parallel, and linked into
``paper_1905_04597_amd/libglbm.so``.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libglbm.so")
ARCH = "gfx950"
LEVELS = (7, 6, 5, 4, 3, 2, 1, 0)  # slowest first; 0 = mixed-level lattices
MIXED_LEVELS = (13, 12, 11, 10, 9, 8)  # the even axis of the mixed lattices beyond 7

FLAGS = [
    "-O3", "-std=c++20", "-fPIC", "--offload-arch=" + ARCH,
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _deps(src: str):
    common = [os.path.join(CSRC, f) for f in ("glbm_device.h", "glbm_internal.h", "glbm_device3.h")]
    if src.endswith("glbm_probe.hip"):
        return [src, os.path.join(os.path.dirname(HERE), "include", "glbm.h")]
    if src.endswith("glbm_api.hip"):
        common.append(os.path.join(os.path.dirname(HERE), "include", "glbm.h"))
    return [src] + common


def _stale(src: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in _deps(src))


def _compile(args):
    src, obj, defines = args
    cmd = [_hipcc(), *FLAGS, *defines, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr[-4000:]))
    return obj


def tasks():
    """(source, object, defines) of every object of the library, slowest first."""
    # the three-dimensional objects are among the slowest: start them first
    out = [(os.path.join(CSRC, "glbm_inst3.hip"), os.path.join(BUILD, "glbm_inst3_%d.o" % k), ["-DGLBM_3D_PART=%d" % k])
             for k in (8, 7, 6, 5, 4, 0, 1, 2, 3)]
    out.append((os.path.join(CSRC, "glbm_api.hip"), os.path.join(BUILD, "glbm_api.o"), []))
    out.append((os.path.join(CSRC, "glbm_probe.hip"), os.path.join(BUILD, "glbm_probe.o"), []))
    for lv in LEVELS:
        for even in (0, 1):
            # one-dimensional; two-dimensional periodic y (or mixed); symmetric with walls
            for compact, walls in ((0, 0), (1, 0), (1, 1)):
                if lv == 0 and (not compact or walls):
                    continue  # the mixed lattices: two-dimensional, one object
                out.append((os.path.join(CSRC, "glbm_inst.hip"),
                              os.path.join(BUILD, "glbm_inst_%s%d%s.o" % ("e" if even else "", lv,
                                                                         ("cw" if walls else "c") if compact else "")),
                              ["-DGLBM_LEVEL=%d" % lv, "-DGLBM_EVEN=%d" % even, "-DGLBM_COMPACT=%d" % compact,
                               "-DGLBM_WALLS=%d" % walls]))
    # levels 8..13: the mixed channel lattice D1Q3 x G-D1Q(2N+2) only
    for lv in MIXED_LEVELS:
        out.insert(2, (os.path.join(CSRC, "glbm_inst.hip"), os.path.join(BUILD, "glbm_inst_e%dc.o" % lv),
                         ["-DGLBM_LEVEL=%d" % lv, "-DGLBM_EVEN=1", "-DGLBM_COMPACT=1"]))
    return out


def build(jobs: int | None = None, incremental: bool = False, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = tasks()
    todo = [t for t in objs if not incremental or _stale(t[0], t[1])]
    jobs = jobs or min(len(todo) or 1, os.cpu_count() or 4, 16)
    if todo:
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            for obj in ex.map(_compile, todo):
                if verbose:
                    print("built", os.path.relpath(obj, HERE), flush=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [t[1] for t in objs]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--incremental", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.incremental, verbose=True))


if __name__ == "__main__":
    sys.exit(main())
