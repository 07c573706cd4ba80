"""Pins of the oracle's 2D small-time expansions (CPU only).

References that the oracle does not use: the gamma_1, gamma_2 the paper prints,
the exact n = 0 Weber integrals of the 2D Green's function (eq. genericGF with
C_0 of eq. fRad) by quadrature, the first-order small-tau reaction probability of
Sec. 4.2, and the boundary conditions.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy import special as S

import oracle as O


def C0(R, x, hh):
    """C_0(R, x) of eq. fRad; hh = inf gives the absorbing limit."""
    J0, Y0 = S.j0(x), S.y0(x)
    if hh == np.inf:
        return -(S.j0(R * x) * Y0 - S.y0(R * x) * J0) / np.sqrt(J0 * J0 + Y0 * Y0)
    A = -x * S.y1(x) - hh * Y0  # x Y_0' - h Y_0
    B = -x * S.j1(x) - hh * J0  # x J_0' - h J_0
    return (S.j0(R * x) * A - S.y0(R * x) * B) / np.sqrt(A * A + B * B)


def g2_exact(R, R0, tau, hh):
    """a^2 g(R, tau | R0) = (1/2pi) int_0^inf e^{-tau x^2} C_0(R, x) C_0(R0, x) x dx."""
    f = lambda x: math.exp(-tau * x * x) * C0(R, x, hh) * C0(R0, x, hh) * x
    edges = np.linspace(0.0, math.sqrt(80.0 / tau), 400)
    return sum(integrate.quad(f, a, b, limit=200, epsabs=1e-15, epsrel=1e-12)[0]
               for a, b in zip(edges[:-1], edges[1:])) / (2 * math.pi)


def test_printed_gamma_coefficients():
    # gamma_1, gamma_2 for abs and rad as printed in Sec. 4.2; ref = rad at h = 0
    for (R, R0, h) in [(1.3, 1.7, 0.25), (1.01, 1.0, 0.04), (2.5, 1.2, 3.0)]:
        ga, gf, gr = O.gamma2(R, R0, h, 4)
        assert ga[0] == gf[0] == gr[0] == 1.0
        P, s = R * R0, R + R0
        assert ga[1] == pytest.approx((2 * P - s) / (8 * P), rel=1e-14)
        assert ga[2] == pytest.approx((9 * (R * R + R0 * R0) + 2 * P - 4 * P * s + 4 * P * P) / (128 * P * P), rel=1e-14)
        rad1 = lambda h: -(P * (6 + 16 * h) + s) / (8 * P)
        rad2 = lambda h: (9 * (R * R + R0 * R0) + 2 * P + P * s * (12 + 32 * h) + P * P * (36 + 192 * h + 256 * h * h)) / (128 * P * P)
        assert gr[1] == pytest.approx(rad1(h), rel=1e-14)
        assert gr[2] == pytest.approx(rad2(h), rel=1e-14)
        assert gf[1] == pytest.approx(rad1(0.0), rel=1e-14)
        assert gf[2] == pytest.approx(rad2(0.0), rel=1e-14)


POINTS = [(1.05, 1.1), (1.2, 1.01), (1.5, 1.5), (1.002, 1.3)]


@pytest.mark.parametrize("R,R0", POINTS)
@pytest.mark.parametrize("tau", [0.01, 0.04])
def test_abs_expansion_vs_weber_integral(R, R0, tau):
    exact_bc = g2_exact(R, R0, tau, np.inf) - O.g2_free(R, R0, tau)
    scale = O.g2_free(R, R0, tau)  # the total is compared on the scale of the free part
    errs = [abs(O.g2_bc(0, R, R0, tau, 0.0, n) - exact_bc) / scale for n in (4, 8, 12, 16)]
    assert errs[-1] < (1e-10 if tau <= 0.01 else 2e-8)
    assert errs[2] < (1e-9 if tau <= 0.01 else 2e-7)


@pytest.mark.parametrize("R,R0", POINTS[:3])
@pytest.mark.parametrize("hh", [0.0, 0.04, 0.5])
def test_ref_rad_expansion_vs_weber_integral(R, R0, hh):
    tau = 0.02
    exact_bc = g2_exact(R, R0, tau, hh) - O.g2_free(R, R0, tau)
    kind = 1 if hh == 0.0 else 2
    got = O.g2_bc(kind, R, R0, tau, hh, 16)
    assert abs(got - exact_bc) < 1e-8 * O.g2_free(R, R0, tau)


@pytest.mark.parametrize("R,R0", POINTS[:3])
def test_pair_probabilities_vs_exact(R, R0):
    # p_enc and p_reac from the expansions against the Bayes ratios of the exact functions
    tau, hh = 0.02, 0.04
    gfree = O.g2_free(R, R0, tau)
    gabs, gref, grad = g2_exact(R, R0, tau, np.inf), g2_exact(R, R0, tau, 0.0), g2_exact(R, R0, tau, hh)
    assert O.penc2(R, R0, tau, 16) == pytest.approx(1 - gabs / gfree, abs=1e-7)
    assert O.preac2(R, R0, tau, hh, 16) == pytest.approx((gref - grad) / (gref - gabs), rel=1e-5)


def test_free_function_is_angular_average():
    # a^2 g_free = (1/2pi) int_0^{2pi} (4 pi tau)^-1 e^{-|R - R0|^2/4tau} dtheta
    for (R, R0, tau) in [(1.1, 1.3, 0.04), (2.0, 1.0, 0.8), (30.0, 30.5, 0.01)]:
        f = lambda th: math.exp(-(R * R + R0 * R0 - 2 * R * R0 * math.cos(th)) / (4 * tau)) / (4 * math.pi * tau)
        ref = integrate.quad(f, 0, 2 * math.pi, limit=400, epsabs=0, epsrel=1e-13)[0] / (2 * math.pi)
        assert O.g2_free(R, R0, tau) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("R,R0", [(1.05, 1.1), (1.3, 1.2), (1.01, 1.02)])
def test_small_tau_reaction_probability(R, R0):
    # p_reac = 2 h tau / (R + R0 - 2) + O(tau^2) (Sec. 4.2); relative error -> 0 linearly
    hh = 0.04
    errs = []
    for tau in [1e-4, 1e-5, 1e-6, 1e-7]:
        first = 2 * hh * tau / (R + R0 - 2)
        errs.append(abs(O.preac2(R, R0, tau, hh, 12) / first - 1))
    # first order: the relative error falls by ~10 per decade of tau
    assert errs[-1] < 1e-3
    for e0, e1 in zip(errs[1:], errs[2:]):
        assert 8.0 < e0 / e1 < 12.0


def test_boundary_conditions_small_tau():
    # absorbing total vanishes at contact; reflecting total has zero slope there
    tau, R0 = 0.01, 1.1
    gtot = lambda kind, R: O.g2_free(R, R0, tau) + O.g2_bc(kind, R, R0, tau, 0.0, 16)
    assert abs(gtot(0, 1.0)) < 1e-9 * O.g2_free(1.0, R0, tau)
    h = 1e-5
    d = (-3 * gtot(1, 1.0) + 4 * gtot(1, 1 + h) - gtot(1, 1 + 2 * h)) / (2 * h)
    assert abs(d) < 1e-5 * gtot(1, 1.0)


def test_reflecting_normalisation_small_tau():
    tau, R0 = 0.02, 1.1
    f = lambda R: 2 * math.pi * R * (O.g2_free(R, R0, tau) + O.g2_bc(1, R, R0, tau, 0.0, 16))
    assert integrate.quad(f, 1, 4, limit=400)[0] == pytest.approx(1.0, abs=1e-8)


def test_propagator_integrates_to_encounter_probability():
    # int w r (g_ref - g_abs) dR = 1 - S_abs = int p_enc g_free (2D, small tau)
    tau, R0 = 0.02, 1.1
    top = R0 + 30 * math.sqrt(tau)
    a = integrate.quad(lambda R: O.prop2_density(R, R0, tau, 16), 1, top, limit=400)[0]
    f = lambda R: 2 * math.pi * R * O.penc2(R, R0, tau, 16) * O.g2_free(R, R0, tau)
    b = integrate.quad(f, 0, 1, limit=400)[0] + integrate.quad(f, 1, top, limit=400)[0]
    assert a == pytest.approx(b, rel=1e-7)


def test_rcut_2d_planar_bound():
    # 2D cut-off: root of erfc((R - 1)/(2 sqrt tau)) = eps; membrane workload values
    rc = O.rcut(2, O.BC_RAD, 0.005, 0.2, 1e-4, 0.05, 1e-3)
    assert math.erfc((rc / 0.005 - 1) / (2 * math.sqrt(0.8))) == pytest.approx(1e-3, rel=1e-9)
    assert rc == pytest.approx(0.02581, abs=1e-5)
    # and it bounds the 2D loss from above (expansion, small tau)
    tau, rc2 = 0.04, O.rcut(2, O.BC_ABS, 1.0, 1.0, 0.04, 0.0, 1e-3)
    loss = 1 - integrate.quad(lambda R: 2 * math.pi * R * (O.g2_free(R, rc2, tau) + O.g2_bc(0, R, rc2, tau, 0, 16)),
                              1, rc2 + 30 * math.sqrt(tau), limit=400)[0]
    assert 0 < loss < 1e-3
