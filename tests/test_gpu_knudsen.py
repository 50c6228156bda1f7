"""The paper's channel setting of sections 5.3-5.4 on the GPU: 200 nodes
across the channel, Knudsen numbers from the slip to the ballistic regime,
the D1Q3 x G-D1Q(2N+2) lattices up to N = 13 (G-D1Q28 x D1Q3).

* One Poiseuille instance per level N in {1, 7, 13} at two Knudsen numbers
  against the FP64 oracle (same step, 1e-5).
* The volumetric flow Q(Kn) of section 5.4 for N in {1, 4, 7, 10, 13}: the
  paper states that the even hierarchy shows the Knudsen minimum from N = 10
  (Fig. 6), and no minimum below; measured here: Q decreasing in Kn for
  N <= 7, a minimum at Kn = 2 for N = 10 and at Kn = 1 for N = 13.  The
  benchmark data (linearised BGK, Cercignani) are not available: agreement
  with the figure's values is parity unpinned; the tests check the oracle
  parity, convergence of the runs and the qualitative claims.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1905_04597_amd import studies

pytestmark = pytest.mark.gpu

NY = 200
KNS = (0.01, 0.03, 0.1, 0.3, 0.5, 1.0, 2.0, 3.33, 10.0)
LEVELS = (1, 4, 7, 10, 13)
STEPS = 40000


def _oracle_poiseuille(N, kn, steps, ny=NY, speed_cs=0.01):
    th = (4 * N + 3) / 3.0
    U = speed_cs * math.sqrt(th)
    nu = th * kn * ny / math.sqrt(2 * th)
    s = oracle.OracleSolver(2, 1, N, 4, ny, kn=kn, bc_y=oracle.BC_WALL, g=8 * nu * U / ny ** 2, even_y=True)
    s.init_fields()
    s.step(steps)
    ux = s.moments()["ux"][:, 0]
    return ux.sum() / (2 * U * ny / 3), ux[0] / ux[ny // 2]


@pytest.mark.parametrize("N", [1, 7, 13])
def test_paper_lattices_match_the_oracle(N):
    steps = 3000
    kns = (0.1, 3.33)
    gpu = {o.kn: o for o in studies.channel_observables("poiseuille", [N], kns, ny=NY, steps=steps)}
    for kn in kns:
        flow, slip = _oracle_poiseuille(N, kn, steps)
        g = gpu[kn]
        print("\n[knudsen] N=%d Kn=%g t=%d flow gpu %.7f oracle %.7f, slip gpu %.7f oracle %.7f"
              % (N, kn, steps, g.flow, flow, g.slip, slip), flush=True)
        assert g.flow == pytest.approx(flow, rel=1e-5)
        assert g.slip == pytest.approx(slip, rel=1e-5)


@pytest.fixture(scope="module")
def sweep():
    out = {}
    for kind in ("poiseuille", "couette"):
        for o in studies.channel_observables(kind, LEVELS, KNS, ny=NY, steps=STEPS):
            out[(kind, o.level, o.kn)] = o
    return out


def test_runs_reach_a_steady_state(sweep):
    worst = max(o.residual for o in sweep.values())
    print("\n[knudsen] worst residual after %d steps: %.2e" % (STEPS, worst), flush=True)
    assert worst < 1e-5


def test_volumetric_flow_over_kn(sweep):
    """The volumetric flow of every level over Kn (printed: the table of
    section 5.4), and the slip regime in which the paper finds all the
    models accurate: at Kn = 0.01 the flow of every level is within 2% of
    the finest level's."""
    table = {}
    for lv in LEVELS:
        table[lv] = [sweep[("poiseuille", lv, kn)].volumetric for kn in KNS]
        print("[knudsen] N=%2d Q(Kn) %s" % (lv, " ".join("%.4f" % q for q in table[lv])), flush=True)
    for lv in LEVELS:
        mins = [i for i in range(1, len(KNS) - 1) if table[lv][i] < table[lv][i - 1] and table[lv][i] < table[lv][i + 1]]
        print("[knudsen] N=%2d interior minimum of Q at Kn %s" % (lv, [KNS[i] for i in mins]), flush=True)
    fine = table[LEVELS[-1]][0]
    for lv in LEVELS:
        assert abs(table[lv][0] - fine) <= 0.02 * fine


def test_knudsen_minimum_from_n10(sweep):
    """Section 5.4: the even hierarchy has no Knudsen minimum at low levels
    (the flow decreases monotonically with Kn) and shows it from N = 10: Q
    falls through the transitional regime and rises again in the ballistic
    one, with the smallest value for 0.5 <= Kn <= 3.33."""
    for lv in LEVELS:
        q = [sweep[("poiseuille", lv, kn)].volumetric for kn in KNS]
        i = int(np.argmin(q))
        if lv <= 7:
            assert all(a > b for a, b in zip(q, q[1:])), (lv, q)
        else:
            assert 0.5 <= KNS[i] <= 3.33 and q[-1] > q[i], (lv, q)
