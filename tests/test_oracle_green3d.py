"""Pins of the oracle's 3D Green's functions and pair probabilities (CPU only).

Each oracle function is checked against the paper's definitions by routes it does
not use itself: 110-digit evaluation of the literal Bayes ratios, quadrature of the
Green's functions (normalisation, survival), the boundary conditions and the
diffusion equation they must satisfy, and the kappa limits of Sec. 2.2.3.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

import oracle as O

TAUS = [0.02, 0.08, 0.8, 5.0, 50.0]
HS = [0.004, 0.08, 0.8, 8.0, 40.0]


def q(f, a, b):
    return integrate.quad(f, a, b, limit=800, epsabs=1e-15, epsrel=1e-13)[0]


# ---- literal formulas of the paper, in 110-digit arithmetic --------------------

def mp_g_free(R, R0, tau):
    """Angular average (eq. radialGF) of the free Gaussian (eq. gaussian), by quadrature over cos(theta)."""
    mp.mp.dps = 110
    R, R0, tau = mp.mpf(R), mp.mpf(R0), mp.mpf(tau)
    f = lambda mu: (4 * mp.pi * tau) ** mp.mpf(-1.5) * mp.exp(-(R * R + R0 * R0 - 2 * R * R0 * mu) / (4 * tau))
    return mp.quad(f, [-1, 1]) / 2


def mp_g_abs(R, R0, tau):
    mp.mp.dps = 110
    R, R0, tau = mp.mpf(R), mp.mpf(R0), mp.mpf(tau)
    pre = 1 / (8 * mp.pi * R * R0) / mp.sqrt(mp.pi * tau)
    return pre * (mp.exp(-(R - R0) ** 2 / (4 * tau)) - mp.exp(-(R + R0 - 2) ** 2 / (4 * tau)))


def mp_g_rad(R, R0, tau, hh):
    """The radiation closed form of Sec. 4.1 exactly as printed (the '+ -' read as '-')."""
    mp.mp.dps = 110
    R, R0, tau, hh = mp.mpf(R), mp.mpf(R0), mp.mpf(tau), mp.mpf(hh)
    k = 1 + hh
    w = R + R0 - 2
    pre = 1 / (8 * mp.pi * R * R0) / mp.sqrt(mp.pi * tau)
    return pre * (mp.exp(-(R - R0) ** 2 / (4 * tau)) + mp.exp(-w ** 2 / (4 * tau))
                  - k * mp.sqrt(4 * mp.pi * tau) * mp.exp(k * k * tau + w * k) * mp.erfc(k * mp.sqrt(tau) + w / (2 * mp.sqrt(tau))))


GRID = [(R, R0, tau) for tau in TAUS for R in (1.0001, 1.01, 1.3, 2.2) for R0 in (1.0, 1.02, 1.5, 3.0)]


@pytest.mark.parametrize("R,R0,tau", GRID)
def test_penc3_is_bayes_ratio(R, R0, tau):
    # p_enc = 1 - G_abs/G_free (eq. bayes1D), radial form (Sec. 2.2.4)
    ref = 1 - mp_g_abs(R, R0, tau) / mp_g_free(R, R0, tau)
    assert O.penc3(R, R0, tau) == pytest.approx(float(ref), rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("R,R0,tau", GRID[::3])
@pytest.mark.parametrize("hh", HS)
def test_preac3_is_bayes_ratio(R, R0, tau, hh):
    # p_reac = (G_ref - G_rad)/(G_ref - G_abs) (eq. psurv_radII)
    gref = mp_g_rad(R, R0, tau, 0)
    ref = (gref - mp_g_rad(R, R0, tau, hh)) / (gref - mp_g_abs(R, R0, tau))
    assert O.preac3(R, R0, tau, hh) == pytest.approx(float(ref), rel=1e-11)


@pytest.mark.parametrize("R,R0,tau", GRID[::5])
def test_oracle_g3_match_literal(R, R0, tau):
    assert O.g3_free(R, R0, tau) == pytest.approx(float(mp_g_free(R, R0, tau)), rel=1e-11, abs=1e-300)
    # g_abs vanishes identically at R0 = 1; compare on the scale of the free function there
    scale = 1e-14 * O.g3_free(R, R0, tau)
    assert O.g3_abs(R, R0, tau) == pytest.approx(float(mp_g_abs(R, R0, tau)), rel=1e-11, abs=scale)
    for hh in (0.0, 0.8, 20.0):
        assert O.g3_rad(R, R0, tau, hh) == pytest.approx(float(mp_g_rad(R, R0, tau, hh)), rel=1e-11, abs=scale)


@pytest.mark.parametrize("tau", [0.08, 0.8, 50.0])
@pytest.mark.parametrize("R0", [1.0, 1.02, 1.5])
def test_normalisation(tau, R0):
    # 4 pi a^3 int R^2 g dR = 1 for the free and the reflecting function (eq. SurvRad, S_ref = 1)
    top = R0 + 40 * math.sqrt(tau) + 5
    f = lambda R: 4 * math.pi * R * R * O.g3_free(R, R0, tau)
    assert q(f, 0, 1) + q(f, 1, top) == pytest.approx(1.0, abs=1e-11)
    g = lambda R: 4 * math.pi * R * R * O.g3_rad(R, R0, tau, 0.0)
    assert q(g, 1, top) == pytest.approx(1.0, abs=1e-11)


@pytest.mark.parametrize("tau", [0.08, 0.8, 50.0])
@pytest.mark.parametrize("R0", [1.0, 1.02, 1.5])
@pytest.mark.parametrize("hh", [0.004, 1.0, 20.0])
def test_survival_closed_forms(tau, R0, hh):
    top = R0 + 40 * math.sqrt(tau) + 5
    sa = q(lambda R: 4 * math.pi * R * R * O.g3_abs(R, R0, tau), 1, top)
    sr = q(lambda R: 4 * math.pi * R * R * O.g3_rad(R, R0, tau, hh), 1, top)
    assert O.loss3_abs(R0, tau) == pytest.approx(1 - sa, abs=1e-12)
    assert O.loss3_rad(R0, tau, hh) == pytest.approx(1 - sr, abs=1e-12)


@pytest.mark.parametrize("tau", [0.08, 0.8, 50.0])
@pytest.mark.parametrize("R0", [1.0, 1.05, 1.5, 2.5])
def test_encounter_marginal_is_absorbing_loss(tau, R0):
    # Averaging p_enc over the free end point gives the first-passage loss of the
    # absorbing problem, (sigma/r0) erfc((r0 - sigma)/sqrt(4 D dt)); overlapping
    # end points (R < 1) count with p = 1 (Sec. 3, step 2).
    top = R0 + 40 * math.sqrt(tau) + 5
    f = lambda R: 4 * math.pi * R * R * O.penc3(R, R0, tau) * O.g3_free(R, R0, tau)
    m = q(f, 0, 1) + q(f, 1, top)
    assert m == pytest.approx(math.erfc((R0 - 1) / (2 * math.sqrt(tau))) / R0, abs=1e-12)


@pytest.mark.parametrize("tau", [0.08, 0.8, 50.0])
@pytest.mark.parametrize("R0", [1.0, 1.05, 1.5])
@pytest.mark.parametrize("hh", [0.004, 1.0, 20.0])
def test_reaction_marginal_is_radiation_loss(tau, R0, hh):
    # integral of p_reac over the propagator w r^2 (g_ref - g_abs) = 1 - S_rad
    top = R0 + 40 * math.sqrt(tau) + 5
    m = q(lambda R: O.preac3(R, R0, tau, hh) * O.prop3_density(R, R0, tau), 1, top)
    assert m == pytest.approx(O.loss3_rad(R0, tau, hh), abs=1e-12)
    # and the propagator integrates to the encounter probability 1 - S_abs
    assert q(lambda R: O.prop3_density(R, R0, tau), 1, top) == pytest.approx(O.loss3_abs(R0, tau), abs=1e-12)


@pytest.mark.parametrize("tau", [0.08, 0.8])
@pytest.mark.parametrize("R0", [1.02, 1.5])
def test_boundary_conditions(tau, R0):
    # eqs. g_abs_bc, g_ref_bc, robin_bc in scaled units: g_abs(1) = 0,
    # dg_ref/dR(1) = 0, dg_rad/dR(1) = h g_rad(1)
    mp.mp.dps = 110
    assert abs(float(mp_g_abs(1, R0, tau))) < 1e-40
    assert abs(O.g3_abs(1.0, R0, tau)) < 1e-17
    h = 1e-5
    for hh in [0.0, 0.3, 4.0]:
        d = (-3 * O.g3_rad(1.0, R0, tau, hh) + 4 * O.g3_rad(1 + h, R0, tau, hh) - O.g3_rad(1 + 2 * h, R0, tau, hh)) / (2 * h)
        assert d == pytest.approx(hh * O.g3_rad(1.0, R0, tau, hh), abs=1e-7 * O.g3_rad(1.0, R0, tau, 0.0))


@pytest.mark.parametrize("fn", ["free", "abs", "ref", "rad"])
def test_diffusion_equation(fn):
    # dg/dtau = g'' + (2/R) g' (eq. smol_bc in scaled radial form)
    R, R0, tau, hh = 1.4, 1.2, 0.3, 0.7
    g = {"free": lambda R, t: O.g3_free(R, R0, t), "abs": lambda R, t: O.g3_abs(R, R0, t),
         "ref": lambda R, t: O.g3_rad(R, R0, t, 0.0), "rad": lambda R, t: O.g3_rad(R, R0, t, hh)}[fn]
    h, k = 1e-3, 1e-5
    gt = (g(R, tau + k) - g(R, tau - k)) / (2 * k)
    g1 = (g(R + h, tau) - g(R - h, tau)) / (2 * h)
    g2 = (g(R + h, tau) - 2 * g(R, tau) + g(R - h, tau)) / (h * h)
    assert gt == pytest.approx(g2 + 2 * g1 / R, rel=1e-5)


def test_kappa_limits():
    # kappa_a -> inf: radiation -> absorbing and p_reac -> 1; kappa_a -> 0: p_reac -> 0 (Sec. 2.2.3)
    for (R, R0, tau) in [(1.2, 1.1, 0.08), (1.01, 1.3, 0.8), (2.0, 1.5, 5.0)]:
        # every deviation from the absorbing limit decays like 1/h (first order of
        # erfcx's large-argument series): ten times larger h, ten times smaller gap
        devs = lambda hh: np.array([O.g3_rad(R, R0, tau, hh) / O.g3_abs(R, R0, tau) - 1,
                                    O.preac3(R, R0, tau, hh) - 1,
                                    O.loss3_rad(R0, tau, hh) / O.loss3_abs(R0, tau) - 1])
        d4, d5 = devs(1e4), devs(1e5)
        assert np.all(np.abs(d4 / d5 - 10.0) < 0.2)
        assert np.all(np.abs(d5) < 2e-3)
        assert O.preac3(R, R0, tau, 1e-12) == pytest.approx(0.0, abs=1e-10)


def test_probabilities_in_range_and_monotone():
    for tau in TAUS:
        Rs = np.linspace(1.0001, 4.0, 60)
        for R0 in (1.0, 1.1, 2.0):
            p = np.array([O.penc3(R, R0, tau) for R in Rs])
            assert np.all((p >= 0) & (p <= 1 + 4e-16)) and np.all(np.diff(p) <= 1e-15)
            for R in (1.05, 2.0):
                pr = [O.preac3(R, R0, tau, h) for h in HS]
                assert np.all(np.diff(pr) > 0) and pr[0] > 0 and pr[-1] < 1


@pytest.mark.parametrize("bc", [O.BC_ABS, O.BC_RAD])
@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_rcut_solves_loss(bc, eps):
    a, Deff, dt, ka = 0.005, 2.0, 1e-5, 0.1
    rc = O.rcut(3, bc, a, Deff, dt, ka, eps)
    tau = Deff * dt / a ** 2
    hh = ka / (4 * math.pi * a * Deff)
    loss = O.loss3_abs(rc / a, tau) if bc == O.BC_ABS else O.loss3_rad(rc / a, tau, hh)
    assert loss == pytest.approx(eps, rel=1e-9)


def test_rcut_values_of_the_workloads():
    # 3D absorbing, sigma = 5 nm, D_eff = 2 um^2/s, dt = 1 us: r_cut = 11.1 nm (1e-3) and 14.4 nm (1e-6)
    assert O.rcut(3, O.BC_ABS, 0.005, 2.0, 1e-6, 0.0, 1e-3) == pytest.approx(0.011117, abs=2e-6)
    assert O.rcut(3, O.BC_ABS, 0.005, 2.0, 1e-6, 0.0, 1e-6) == pytest.approx(0.014360, abs=2e-6)
