"""Pins of the oracle's equilibrium (section 2, section 3, Appendices A and B).

Each check compares the oracle's closed form (Eq. maineq03) with something
the paper or the mathematics fixes independently of it: the worked example
of Appendix A, the printed D1Q3 root model, exact rational convolution
powers, brute-force enumeration of the 3^N outcomes of the dice problem, the
moment identities of section 3 / Appendix B and the product form of the
moment generating function (Eq. mgf).
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_fixture(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


# ---------------------------------------------------------------- App. A
def test_appendix_a_worked_example():
    """G-D1Q5 at unit temperature, c = sqrt(3/2): printed products of P+, P0, P-."""
    rows = _read_fixture("appendix_a_g_d1q5.txt")
    csq = float(Fraction([r for r in rows if r[0] == "csq"][0][1]))
    c = math.sqrt(csq)
    terms = [r for r in rows if r[0] == "term"]
    for u in (-0.4, -0.07, 0.0, 0.013, 0.25, 0.9):
        Pp = (1 + c * u + u * u / 2) / (4 * csq)
        Pm = (1 - c * u + u * u / 2) / (4 * csq)
        P0 = 1 - Pp - Pm
        want = np.zeros(5)
        for _, n, coef, ep, e0, em in terms:
            want[int(n) + 2] += int(coef) * Pp ** int(ep) * P0 ** int(e0) * Pm ** int(em)
        got = oracle.equilibrium_1d(2, u, c=c, theta0=1.0)
        np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-16)


def test_appendix_a_rest_weights():
    rows = _read_fixture("appendix_a_g_d1q5.txt")
    want = np.zeros(5)
    for _, n, v in [r for r in rows if r[0] == "rest"]:
        want[int(n) + 2] = float(Fraction(v))
    # the rest state does not depend on the unit system
    np.testing.assert_allclose(oracle.rest_weights(2), want, rtol=1e-15)
    np.testing.assert_allclose(oracle.equilibrium_1d(2, 0.0, c=math.sqrt(1.5), theta0=1.0), want, rtol=1e-15)


def test_d1q3_root_model():
    """N = 1 reduces to the printed D1Q3 equilibrium of section 2."""
    rows = _read_fixture("d1q3_equilibrium.txt")
    for c in (1.0, math.sqrt(3.0), 0.7):
        for u in (-0.3, -0.01, 0.0, 0.05, 0.2):
            v = u / c
            want = np.zeros(3)
            for _, n, a0, a1, a2 in rows:
                want[int(n) + 1] = float(Fraction(a0)) + float(Fraction(a1)) * v + float(Fraction(a2)) * v * v
            got = oracle.equilibrium_1d(1, u, c=c, theta0=c * c / 3.0)
            np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-16)


# ------------------------------------------------- exact rational weights
def _poly_power(p, N):
    out = [Fraction(1)]
    for _ in range(N):
        nxt = [Fraction(0)] * (len(out) + len(p) - 1)
        for i, x in enumerate(out):
            for j, y in enumerate(p):
                nxt[i + j] += x * y
        out = nxt
    return out


@pytest.mark.parametrize("N", range(1, 8))
def test_rest_weights_are_convolution_powers(N):
    """W_n = coefficients of (1/6 z^-1 + 2/3 + 1/6 z)^N (N-fold sum of D1Q3 at rest)."""
    want = _poly_power([Fraction(1, 6), Fraction(2, 3), Fraction(1, 6)], N)
    assert sum(want) == 1
    np.testing.assert_allclose(oracle.rest_weights(N), [float(w) for w in want], rtol=2e-15)


# ------------------------------------------------------- brute force 3^N
def _enumerate(N, u, c, theta0):
    """Law of the sum of N i.i.d. steps in {-c, 0, c}, mean u/N, variance theta0/N.

    The step probabilities follow from those two conditions alone
    (section 2, the triangular-array construction), not from Eq. maineq04."""
    mean = u / N
    second = theta0 / N + mean * mean
    pp = 0.5 * (second / c ** 2 + mean / c)
    pm = 0.5 * (second / c ** 2 - mean / c)
    p = {-1: pm, 0: 1.0 - pp - pm, 1: pp}
    out = np.zeros(2 * N + 1)
    for steps in itertools.product((-1, 0, 1), repeat=N):
        prob = 1.0
        for s in steps:
            prob *= p[s]
        out[sum(steps) + N] += prob
    return out


@pytest.mark.parametrize("N", range(1, 8))
def test_closed_form_equals_enumeration(N):
    for theta0 in (1.0, N / 3.0):
        c = math.sqrt(3 * theta0 / N)
        for u in (-0.5, -0.1, 0.0, 0.02, 0.3, 0.8):
            np.testing.assert_allclose(oracle.equilibrium_1d(N, u, c=c, theta0=theta0),
                                       _enumerate(N, u, c, theta0), rtol=1e-13, atol=1e-17)


def test_step_probabilities_match_definition():
    for N in range(1, 8):
        for u in (-0.2, 0.0, 0.1):
            pm, p0, pp = oracle.step_probabilities(N, u)
            # mean and variance of one step in lattice units (c = 1, theta0 = N/3)
            assert pp - pm == pytest.approx(u / N, abs=1e-15)
            assert (pp + pm) - (u / N) ** 2 == pytest.approx((N / 3.0) / N, abs=1e-15)
            assert pm + p0 + pp == pytest.approx(1.0, abs=1e-15)


# ------------------------------------------------------- moment identities
def _moments(N, u, theta0=1.0, kmax=8):
    c = math.sqrt(3 * theta0 / N)
    F = oracle.equilibrium_1d(N, u, c=c, theta0=theta0)
    v = np.arange(-N, N + 1) * c
    return [float((F * v ** k).sum()) for k in range(kmax + 1)]


def _maxwell(k, u, theta):
    """E[(u + sqrt(theta) Z)^k] for a standard normal Z."""
    s = 0.0
    for j in range(0, k + 1, 2):
        dfact = math.prod(range(j - 1, 0, -2)) if j > 0 else 1
        s += math.comb(k, j) * u ** (k - j) * theta ** (j / 2) * dfact
    return s


@pytest.mark.parametrize("N", range(1, 8))
def test_exact_moments_orders_0_to_2(N):
    """Density, momentum and momentum flux are those of the Maxwellian (section 2)."""
    for theta0 in (1.0, 0.5):
        for u in (-0.3, 0.0, 0.1, 0.7):
            m = _moments(N, u, theta0)
            assert abs(m[0] - 1.0) <= 1e-14
            assert abs(m[1] - u) <= 1e-14
            assert abs(m[2] - (u * u + theta0)) <= 1e-13


@pytest.mark.parametrize("N", range(1, 8))
def test_third_moment_error(N):
    """Section 3 and Appendix B: Maxwell minus model third moment is u^3 / N^2."""
    theta0 = 1.0
    for u in (-0.6, -0.1, 0.05, 0.4, 1.0):
        m3 = _moments(N, u, theta0)[3]
        assert _maxwell(3, u, theta0) - m3 == pytest.approx(u ** 3 / N ** 2, rel=1e-11, abs=1e-15)
        # the factorial-moment expansion printed in Appendix B
        c = math.sqrt(3 * theta0 / N)
        pm, _, pp = oracle.step_probabilities(N, u, c=c, theta0=theta0)
        d, s = (pp - pm) * c, (pp + pm) * c * c
        ab = N * (N - 1) * (N - 2) * d ** 3 + 3 * N * (N - 1) * d * s + N * (pp - pm) * c ** 3
        assert ab == pytest.approx(m3, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("N", range(1, 8))
def test_fourth_moment_error_corrected(N):
    """Fourth moment: model - Maxwell = -3 theta u^2 / N^2 - (4N - 3) u^4 / N^3.

    Both printed forms (section 3 and Appendix B) are inconsistent with each
    other and with N = 1; this corrected form is the one that the MGF of
    Eq. mgf gives (derived symbolically) and that D1Q3 satisfies exactly."""
    theta0 = 1.0
    for u in (-0.6, -0.1, 0.05, 0.4, 1.0):
        m4 = _moments(N, u, theta0)[4]
        want = -3 * theta0 * u ** 2 / N ** 2 - (4 * N - 3) * u ** 4 / N ** 3
        assert m4 - _maxwell(4, u, theta0) == pytest.approx(want, rel=1e-10, abs=1e-14)


def test_fourth_moment_d1q3_direct():
    """For D1Q3 the velocities are -c, 0, c so m4 = c^2 m2 exactly."""
    for u in (0.0, 0.1, 0.5):
        c = math.sqrt(3.0)
        m = _moments(1, u, 1.0)
        assert m[4] == pytest.approx(c * c * m[2], rel=1e-13)
        assert m[4] - _maxwell(4, u, 1.0) == pytest.approx(-3 * u * u - u ** 4, abs=1e-12)


@pytest.mark.parametrize("N", range(1, 8))
def test_mgf_product_form(N):
    """Eq. mgf: sum_n e^{n c s} F_n = (P- e^{-cs} + P0 + P+ e^{cs})^N."""
    theta0 = 1.0
    c = math.sqrt(3 * theta0 / N)
    for u in (-0.3, 0.0, 0.2):
        F = oracle.equilibrium_1d(N, u, c=c, theta0=theta0)
        pm, p0, pp = oracle.step_probabilities(N, u, c=c, theta0=theta0)
        for s in (-1.3, -0.2, 0.05, 0.7, 2.0):
            lhs = float((F * np.exp(np.arange(-N, N + 1) * c * s)).sum())
            rhs = (pm * math.exp(-c * s) + p0 + pp * math.exp(c * s)) ** N
            assert lhs == pytest.approx(rhs, rel=1e-13)


@pytest.mark.parametrize("N", range(1, 8))
def test_log_mgf_cumulants(N):
    """log M(s) = u s + theta s^2/2 + O(1/N^2): third and fourth cumulants.

    Corrected coefficients of the expansion printed in section 3:
    s^3: -u^3/(6 N^2) (cumulant -u^3/N^2), s^4: u^2 (u^2 - N theta)/(8 N^3)
    (cumulant 3 u^2 (u^2 - N theta)/N^3)."""
    theta0 = 1.0
    for u in (-0.4, 0.1, 0.6):
        m = _moments(N, u, theta0, kmax=4)
        k2 = m[2] - m[1] ** 2
        k3 = m[3] - 3 * m[2] * m[1] + 2 * m[1] ** 3
        k4 = m[4] - 4 * m[3] * m[1] - 3 * m[2] ** 2 + 12 * m[2] * m[1] ** 2 - 6 * m[1] ** 4
        assert k2 == pytest.approx(theta0, rel=1e-12)
        assert k3 == pytest.approx(-u ** 3 / N ** 2, rel=1e-9, abs=1e-14)
        assert k4 == pytest.approx(3 * u * u * (u * u - N * theta0) / N ** 3, rel=1e-9, abs=1e-13)


def test_highest_moment_errors_decrease_with_N():
    """Section 1/3: the errors of all higher moments shrink monotonically in N."""
    theta0 = 1.0
    for u in np.linspace(0.02, math.sqrt(2 * theta0), 12):
        for k in range(3, 9):
            errs = [abs(_moments(N, u, theta0)[k] - _maxwell(k, u, theta0)) for N in range(1, 8)]
            assert all(errs[i] > errs[i + 1] for i in range(len(errs) - 1)), (u, k, errs)


@pytest.mark.parametrize("N", range(1, 8))
def test_weights_sum_to_one_at_any_velocity(N):
    for u in np.linspace(-N * 0.8, N * 0.8, 9):
        assert oracle.equilibrium_1d(N, float(u)).sum() == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("N", range(1, 8))
def test_positivity_domain(N):
    """Section 3: the equilibrium is non-negative iff |u| <= sqrt(2 N theta0)."""
    for theta0 in (1.0, N / 3.0):
        c = math.sqrt(3 * theta0 / N)
        edge = math.sqrt(2 * N * theta0)
        inside = oracle.equilibrium_1d(N, 0.999 * edge, c=c, theta0=theta0)
        assert inside.min() >= 0.0
        pm, p0, pp = oracle.step_probabilities(N, 1.001 * edge, c=c, theta0=theta0)
        assert p0 < 0.0 and pm >= 0.0 and pp >= 0.0


def test_tau_from_kn_matches_mean_free_path_route():
    """Section 5.2: k = sqrt(pi/(2 theta)) nu / H, delta = sqrt(pi)/(2k), Kn = 1/delta."""
    for kn, H, theta in ((0.01, 2000, 1.0), (0.1, 1024, 5 / 3), (10.0, 256, 1.0), (0.3, 64, 1 / 3)):
        tau = oracle.tau_from_kn(kn, H, theta)
        nu = theta * tau
        k = math.sqrt(math.pi / (2 * theta)) * nu / H
        delta = math.sqrt(math.pi) / (2 * k)
        assert 1.0 / delta == pytest.approx(kn, rel=1e-14)
