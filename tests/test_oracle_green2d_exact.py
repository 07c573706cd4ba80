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
