"""Write the long-run reference results of the FP64 oracle (tests/golden/*.npz).

Calls only ``oracle/``.  Channel flows with periodic x and x-uniform data keep
every column identical in the oracle, so each reference is computed on a
single column (nx = 1) and holds per-row moments.

    python tests/golden/make_golden.py [--only NAME]

Files:
  poiseuille_d2q121_ny1024_t20000.npz  G-D2Q(11x11), ny = 1024, Kn = 0.1,
                                        g = 1e-5, walls at rest, from rest,
                                        moments at t = 2000 and t = 20000
  couette_d2q49_ny256_kn<Kn>.npz        G-D2Q(7x7), ny = 256, walls at -/+0.1 c_s
                                        (c_s = 1 at N = 3), from rest, run until
                                        the residual ||u(t)-u(t-1)|| / ||u(t)||
                                        falls below 1e-10 (checked every 100 steps)
"""
import argparse
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def moments_col(s):
    m = s.moments()
    return {k: v[:, 0].copy() for k, v in m.items()}


def poiseuille():
    s = oracle.OracleSolver(2, 5, 5, 1, 1024, kn=0.1, bc_y=oracle.BC_WALL, g=1e-5)
    s.init_fields()
    out = {}
    t0 = time.time()
    s.step(2000)
    for k, v in moments_col(s).items():
        out["t2000_" + k] = v
    s.step(18000)
    for k, v in moments_col(s).items():
        out["t20000_" + k] = v
    st = s.stats()
    for k, v in st.items():
        out["t20000_stat_" + k] = np.float64(v)
    out["tau"] = np.float64(s.tau)
    path = os.path.join(HERE, "poiseuille_d2q121_ny1024_t20000.npz")
    np.savez_compressed(path, **out)
    print("wrote %s (%.0f s)" % (path, time.time() - t0), flush=True)


def couette(kn):
    U = 0.1 * math.sqrt(3 / 3.0)
    s = oracle.OracleSolver(2, 3, 3, 1, 256, kn=kn, bc_y=oracle.BC_WALL, wall_u=(-U, U))
    s.init_fields()
    t0 = time.time()
    steps = 0
    res = float("nan")
    while steps < 2_000_000:
        s.step(100)
        steps += 100
        res = s.stats()["residual"]
        if res < 1e-10:
            break
    out = {k: v for k, v in moments_col(s).items()}
    for k, v in s.stats().items():
        out["stat_" + k] = np.float64(v)
    out["steps"] = np.int64(steps)
    out["tau"] = np.float64(s.tau)
    out["wall_u"] = np.float64(U)
    path = os.path.join(HERE, "couette_d2q49_ny256_kn%g.npz" % kn)
    np.savez_compressed(path, **out)
    print("wrote %s: %d steps, residual %.2e (%.0f s)" % (path, steps, res, time.time() - t0), flush=True)


JOBS = {"poiseuille": poiseuille}
for _kn in (0.01, 0.1, 1.0, 10.0):
    JOBS["couette_kn%g" % _kn] = (lambda kn: (lambda: couette(kn)))(_kn)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None)
    a = ap.parse_args()
    for name, job in JOBS.items():
        if a.only is None or a.only == name:
            job()


if __name__ == "__main__":
    main()
