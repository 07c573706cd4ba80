"""Pins of the oracle's exact 2D radial functions (quadrature of the n = 0 term of the 2D
Green's function, eqs. genericGF and fRad), which take over from the small-time expansions
beyond their regime (CPU only).

References the oracle does not use: scipy's adaptive quadrature with scipy's Bessel functions
(the Weber integral of test_oracle_green2d), the small-time expansions where they hold, the
boundary conditions, normalisation, the kappa -> infinity limit and derivatives by finite
differences.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O

from .test_oracle_green2d import g2_exact

TAUS = [0.04, 0.8, 5.0]


@pytest.mark.parametrize("tau", TAUS)
@pytest.mark.parametrize("R,R0", [(1.02, 1.3), (1.7, 1.1), (3.0, 4.5)])
def test_weber_integrals_against_scipy(R, R0, tau):
    hh = 0.04
    got = O.g2x(R, R0, tau, hh)
    for kind, h in ((0, np.inf), (1, 0.0), (2, hh)):
        ref = g2_exact(R, R0, tau, h)
        assert got[kind] == pytest.approx(ref, rel=1e-9, abs=1e-13 * O.g2_free(R, R0, tau)), kind


@pytest.mark.parametrize("R,R0", [(1.05, 1.1), (1.2, 1.01), (1.5, 1.5), (1.002, 1.3)])
def test_small_tau_agrees_with_the_expansions(R, R0):
    # at tau = 0.01 the order-16 expansions hold to ~1e-10 of the free function
    tau, hh = 0.01, 0.3
    got = O.g2x(R, R0, tau, hh)
    gf = O.g2_free(R, R0, tau)
    for kind in range(3):
        exp_total = gf + O.g2_bc(kind, R, R0, tau, hh, 16)
        assert abs(got[kind] - exp_total) < 1e-10 * gf, kind
    assert O.penc2x(R, R0, tau) == pytest.approx(O.penc2(R, R0, tau, 16), abs=1e-9)
    # p_reac is a ratio of boundary parts: it is well conditioned for quadrature only where they
    # are not negligible against the free part (at (1.5, 1.5) they are e^-25 of it)
    if abs(got[1] - gf) > 1e-6 * gf:
        assert O.preac2x(R, R0, tau, hh) == pytest.approx(O.preac2(R, R0, tau, hh, 16), rel=1e-7)


@pytest.mark.parametrize("tau", TAUS)
def test_boundary_conditions(tau):
    # absorbing: g = 0 at contact; reflecting: dg/dR = 0; radiation: dg/dR = h g (eq. robin_bc,
    # reduced units); one-sided second-order differences
    R0, hh, e = 1.4, 0.7, 1e-4
    g = lambda R: O.g2x(R, R0, tau, hh)
    g1, g2, g3 = g(1.0), g(1.0 + e), g(1.0 + 2 * e)
    scale = O.g2_free(1.0, R0, tau)
    assert abs(g1[0]) < 1e-12 * scale
    d = (-3 * g1 + 4 * g2 - g3) / (2 * e)
    assert abs(d[1]) < 1e-6 * scale
    assert d[2] == pytest.approx(hh * g1[2], rel=1e-6)


@pytest.mark.parametrize("tau", TAUS)
def test_reflecting_mass_is_one_and_absorbing_mass_is_survival(tau):
    R0 = 1.3
    top = R0 + 12 * math.sqrt(tau) + 1
    m = O.m2x(top, R0, tau)
    assert m[1] == pytest.approx(1.0, abs=1e-11)  # a reflecting disk loses nothing
    assert 0.0 < m[0] < m[1]
    # the absorbing mass is the survival, 1 - int p_enc g_free over the whole plane (eq. laplaceAnsatz)
    f = lambda R: 2 * math.pi * R * (1 - O.penc2x(R, R0, tau)) * O.g2_free(R, R0, tau)
    surv = integrate.quad(f, 1.0, top, limit=200, epsabs=1e-12)[0]
    assert m[0] == pytest.approx(surv, abs=1e-8)


def test_mass_derivative_is_the_radial_density():
    tau, R0, R, e = 0.8, 1.6, 2.1, 1e-4
    gp, gm = O.m2x(R + e, R0, tau), O.m2x(R - e, R0, tau)
    g = O.g2x(R, R0, tau, 0.0)
    d = (gp - gm) / (2 * e)
    assert d[0] == pytest.approx(2 * math.pi * R * g[0], rel=1e-7)
    assert d[1] == pytest.approx(2 * math.pi * R * g[1], rel=1e-7)


def test_large_kappa_limit_is_absorbing():
    for (R, R0, tau) in [(1.1, 1.4, 0.8), (2.0, 1.2, 0.04)]:
        g = O.g2x(R, R0, tau, 1e8)
        assert g[2] == pytest.approx(g[0], rel=1e-6, abs=1e-10 * O.g2_free(R, R0, tau))


@pytest.mark.parametrize("tau", [0.04, 0.8])
def test_pair_probabilities_are_probabilities(tau):
    rng = np.random.default_rng(3)
    for _ in range(6):
        R, R0 = 1 + rng.exponential(2 * math.sqrt(tau)), 1 + rng.exponential(2 * math.sqrt(tau))
        p = O.penc2x(R, R0, tau)
        q = O.preac2x(R, R0, tau, 0.04)
        assert 0.0 <= p <= 1.0 and 0.0 <= q <= 1.0
    assert O.penc2x(1.0 + 1e-9, 1.5, tau) == pytest.approx(1.0, abs=1e-6)
    assert O.penc2x(0.9, 1.5, tau) == 1.0


@pytest.mark.parametrize("R0", [1.0, 1.3, 4.0])
def test_inversion_sampler(R0):
    # R''(u) solves M(R'') = u M(top) with M the reflecting-minus-absorbing mass; it increases with u
    tau = 0.8
    top = R0 + 12 * math.sqrt(tau) + 1
    mt = O.m2x(top, R0, tau)
    prev = 1.0
    for u in (1e-6, 0.1, 0.5, 0.9, 0.999999):
        Rp = O.sample_prop2x(R0, tau, u)
        assert 1.0 <= Rp <= top and Rp > prev
        m = O.m2x(Rp, R0, tau)
        assert (m[1] - m[0]) == pytest.approx(u * (mt[1] - mt[0]), rel=1e-10, abs=1e-12)
        prev = Rp


def test_large_h_reaction_probability():
    # large intrinsic rates, where the q^-1 small-time series fails (p_reac from it is ~1e4 at
    # h = 20): the exact p_reac is a probability, rises with h towards 1 (the absorbing limit)
    # and equals the Bayes ratio of scipy's Weber integrals
    tau, R, R0 = 0.04, 1.05, 1.1
    prev = 0.0
    for hh in (0.5, 2.0, 20.0, 200.0):
        p = O.preac2x(R, R0, tau, hh)
        assert prev < p <= 1.0
        prev = p
    gabs, gref, grad = g2_exact(R, R0, tau, np.inf), g2_exact(R, R0, tau, 0.0), g2_exact(R, R0, tau, 20.0)
    assert O.preac2x(R, R0, tau, 20.0) == pytest.approx((gref - grad) / (gref - gabs), rel=1e-7)
    assert O.preac2x(R, R0, tau, 1e7) == pytest.approx(1.0, abs=1e-5)
    assert abs(O.preac2(R, R0, tau, 20.0, 12)) > 10  # the expansion is useless there


# ---------------------------------------------------------------------------
# An independent reference beyond the quadrature's floor: the boundary parts of
# the 2D radial Green's function in the Laplace domain (Sec. 4.2, eqs. absPert,
# refPert, radPert; reduced units a = 1, D = 1) inverted numerically on Talbot's
# contour (mpmath).  They are computed without subtracting the free part, so
# they keep their relative precision where the x quadrature, which sums O(1)
# oscillating terms to a result of size e^{-(R+R0-2)^2/4tau}, cannot.
# ---------------------------------------------------------------------------
def _laplace_probs(R, R0, tau, hh):
    import mpmath as mp

    mp.mp.dps = 15

    def inv(kind):
        def f(p):
            q = mp.sqrt(p)
            if kind == 0:
                ratio = mp.besseli(0, q) / mp.besselk(0, q)
            elif kind == 1:
                ratio = -mp.besseli(1, q) / mp.besselk(1, q)
            else:
                ratio = (hh / q * mp.besseli(0, q) - mp.besseli(1, q)) / (hh / q * mp.besselk(0, q) + mp.besselk(1, q))
            return -ratio * mp.besselk(0, q * R0) * mp.besselk(0, q * R) / (2 * mp.pi)

        return mp.invertlaplace(f, tau, method="talbot")

    ga, gr, gd = inv(0), inv(1), inv(2)
    gf = mp.exp(-(R * R + R0 * R0) / (4 * tau)) * mp.besseli(0, R * R0 / (2 * tau)) / (4 * mp.pi * tau)  # Weber
    return float(-ga / gf), float((gr - gd) / (gr - ga))


def test_laplace_reference_agrees_with_scipy_quadrature():
    # the reference itself, where scipy's quadrature resolves the boundary parts
    R, R0, tau, hh = 1.05, 1.1, 0.04, 0.8
    pe, pr = _laplace_probs(R, R0, tau, hh)
    gf = O.g2_free(R, R0, tau)
    ga, gr, gd = g2_exact(R, R0, tau, np.inf), g2_exact(R, R0, tau, 0.0), g2_exact(R, R0, tau, hh)
    assert pe == pytest.approx(1.0 - ga / gf, abs=1e-9)
    assert pr == pytest.approx((gr - gd) / (gr - ga), abs=1e-9)


@pytest.mark.slow
@pytest.mark.parametrize("tau,tol", [(0.2, 1e-6), (0.5, 1e-6), (0.8, 1.5e-6)])
def test_exact_mode_on_both_sides_of_its_switch(tau, tol):
    # The exact 2D mode evaluates pairs with R0 <= x2_switch(tau) by quadrature and farther out
    # by the order-12 expansion.  Just inside the switch and sqrt(tau) beyond it, both hold
    # p_enc and p_reac to 1e-6 for tau <= 0.5 and to 1.5e-6 at tau = 0.8 near contact, where
    # the expansion is weakest (h = 0.8, larger than the membrane workload's 0.04).
    sw = O.x2_switch(tau)
    assert sw == pytest.approx(1.0 + (8.4 if tau <= 0.5 else 9.0) * math.sqrt(tau))
    hh = 0.8
    for R0 in (sw - 0.5 * math.sqrt(tau), sw + math.sqrt(tau)):
        for R in (1.0005, 1.3):
            pe, pr = _laplace_probs(R, R0, tau, hh)
            if R0 <= sw:
                got = O.penc2x(R, R0, tau), O.preac2x(R, R0, tau, hh)
            else:
                got = O.penc2(R, R0, tau, 12), O.preac2(R, R0, tau, hh, 12)
            assert abs(got[0] - pe) <= tol, (R, R0, got[0], pe)
            assert abs(got[1] - pr) <= tol, (R, R0, got[1], pr)


@pytest.mark.slow
@pytest.mark.parametrize("n,tau", [(8, 0.03), (12, 0.05)])
def test_expansion_holds_1e6_up_to_its_tau_limit(n, tau):
    # The library accepts the order-n expansion up to a tau that grows with n (8: 0.03,
    # 12: 0.05; beyond it sim_create refuses the handle): at that limit it holds p_enc and
    # p_reac to 1e-6 at contact, where it is weakest, and three orders fewer do not.
    hh = 0.8
    worst, worst_lower = 0.0, 0.0
    for R, R0 in ((1.0005, 1.0005), (1.02, 1.1)):
        pe, pr = _laplace_probs(R, R0, tau, hh)
        worst = max(worst, abs(O.penc2(R, R0, tau, n) - pe), abs(O.preac2(R, R0, tau, hh, n) - pr))
        worst_lower = max(worst_lower, abs(O.penc2(R, R0, tau, n - 3) - pe), abs(O.preac2(R, R0, tau, hh, n - 3) - pr))
    assert worst <= 1e-6
    assert worst_lower > 1e-6
