"""Pins of the oracle's 2D angular propagator (CPU only).

On a membrane the propagated pair's angle theta to its old separation is drawn from
r (G_ref - G_abs) (Sec. 3, Details, J = r) with the cos(n theta) series of eq. genericGF for
the reflecting (h -> 0) and absorbing (h -> infinity) circles, eq. fRad.  The pins:
  - the integer-order Bessel functions against scipy's;
  - the n = 0 coefficient against the exact 2D radial functions (w_0 = 2 pi (g_ref - g_abs),
    the quadrature of the exact 2D section, itself pinned against the small-time expansions);
  - the same functions and rule on the free Green's function against Weber's integral,
    int e^{-tau x^2} J_n(Rx) J_n(R0x) x dx = e^{-(R^2+R0^2)/4tau} I_n(R R0/2tau) / (2 tau);
  - the locally flat circle (tau -> 0 near contact): the lateral step of the reflected part is
    Gaussian with variance 2 tau, P(|theta| > t) -> erfc(t sqrt(R R0) / (2 sqrt(tau)));
  - a Monte Carlo of reflected Brownian motion in the plane at tau = 0.5 (E[cos n theta] in
    two radius windows);
  - the distribution function runs from 0 to 1, is monotone, and the draw inverts it.
"""
import ctypes
import math

import numpy as np
import pytest
from scipy import special as sp

import oracle as O


@pytest.mark.parametrize("z", [1e-3, 0.05, 0.7, 5.0, 40.0, 300.0])
def test_integer_order_bessel_functions(z):
    kmax = 161
    J, Y = O.bessel_int(kmax, z)
    n = np.arange(kmax + 1) - 1
    Jr, Yr = sp.jv(n, z), sp.yv(n, z)
    scale = math.sqrt(2.0 / (math.pi * z))
    ok = np.abs(Jr) > 1e-280
    tol = 1e-12 if z < 100 else 5e-10  # scipy's own accuracy at large arguments
    assert np.all(np.abs(J[ok] - Jr[ok]) <= tol * np.maximum(np.abs(Jr[ok]), 1e-6 * scale))
    ok = np.abs(Yr) < 1e300
    tol = 2e-12 if z < 100 else 5e-11
    assert np.all(np.abs(Y[ok] - Yr[ok]) <= tol * np.maximum(np.abs(Yr[ok]), 1e-6 * scale))


CASES = [(1.5, 1.2, 0.8), (1.05, 1.0, 0.04), (1.3, 1.25, 0.008), (1.0, 1.6, 0.3), (1.2, 1.1, 0.04)]


@pytest.mark.parametrize("R,R0,tau", CASES)
def test_zeroth_coefficient_is_the_exact_radial_function(R, R0, tau):
    w = O.angle2_coef(0, R, R0, tau)
    g = np.zeros(3)
    O.lib().orc_g2x(R, R0, tau, 0.0, g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    want = 2.0 * math.pi * (g[1] - g[0])
    # both sides are quadratures of terms that cancel down to the image term
    assert abs(w[0] - want) <= (1e-13 + 1e-15 * math.exp((R + R0 - 2.0) ** 2 / (4.0 * tau))) * abs(want) * 10


@pytest.mark.parametrize("R,R0,tau", CASES)
def test_free_space_terms_match_webers_integral(R, R0, tau):
    w = O.angle2_coef(1, R, R0, tau)
    n = np.arange(len(w))
    want = math.exp(-(R - R0) ** 2 / (4.0 * tau)) / (2.0 * tau) * sp.ive(n, R * R0 / (2.0 * tau))
    assert np.all(np.abs(w - want) <= 1e-12 * want[0])


@pytest.mark.parametrize("a,b", [(0.5, 0.8), (0.0, 1.0), (1.0, 0.2)])
def test_locally_flat_circle_gives_a_gaussian_lateral_step(a, b):
    tau = 2e-3
    s = math.sqrt(tau)
    R0, R = 1.0 + a * s, 1.0 + b * s
    w = O.angle2_coef(0, R, R0, tau)
    for t in (0.5 * s, s, 2.0 * s, 3.0 * s):
        tail = 1.0 - O.angle2_cdf(w, t)
        assert abs(tail - math.erfc(t * math.sqrt(R * R0) / (2.0 * s))) < 0.006


def _reflected_paths(R0, tau, M, npath, seed):
    """End radius and cos theta of the planar paths that met the circle (sub-steps of variance
    2 tau / M per coordinate, mirrored across the circle when they end inside it, contacts in
    between from the flat-surface bridge probability)."""
    rng = np.random.default_rng(seed)
    x = np.zeros((npath, 2))
    x[:, 0] = R0
    r = np.full(npath, R0)
    hit = np.zeros(npath, bool)
    dt = tau / M
    for _ in range(M):
        y = x + math.sqrt(2.0 * dt) * rng.standard_normal((npath, 2))
        ry = np.linalg.norm(y, axis=1)
        inside = ry < 1.0
        pc = np.exp(-np.maximum(r - 1.0, 0.0) * np.maximum(ry - 1.0, 0.0) / dt)
        hit |= inside | (rng.random(npath) < pc)
        y[inside] *= ((2.0 - ry[inside]) / ry[inside])[:, None]
        ry[inside] = 2.0 - ry[inside]
        x, r = y, ry
    return r[hit], x[hit, 0] / r[hit]


def test_angular_moments_match_reflected_brownian_motion():
    R0, tau = 1.2, 0.5
    r, c = _reflected_paths(R0, tau, 300, 100000, 3)
    xg, wg = np.polynomial.legendre.leggauss(12)
    for lo, hi in ((1.0, 1.3), (1.3, 1.7)):
        sel = (r >= lo) & (r < hi)
        n = sel.sum()
        Rs = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
        W = np.array([O.angle2_coef(0, Rv, R0, tau, 4) for Rv in Rs])
        m = (wg[:, None] * Rs[:, None] * W).sum(0)  # the radial weight of the window is r w_0
        th = np.arccos(np.clip(c[sel], -1.0, 1.0))
        for k in (1, 2):
            v = np.cos(k * th)
            err = v.std() / math.sqrt(n)
            assert abs(v.mean() - m[k] / m[0]) < 4.0 * err + 0.006, (lo, k, v.mean(), m[k] / m[0])


@pytest.mark.parametrize("R,R0,tau", CASES)
def test_distribution_function_and_its_inverse(R, R0, tau):
    w = O.angle2_coef(0, R, R0, tau)
    ts = np.linspace(0.0, math.pi, 801)
    F = np.array([O.angle2_cdf(w, t) for t in ts])
    assert abs(F[0]) < 1e-15 and abs(F[-1] - 1.0) < 1e-12
    assert np.min(np.diff(F)) > -1e-12
    for u in (1e-6, 0.2, 0.5, 0.93, 1.0 - 1e-9):
        t = O.sample_angle2(R, R0, tau, u)
        assert 0.0 <= t <= math.pi
        assert abs(O.angle2_cdf(w, t) - u) < 1e-12


def test_out_of_range_pairs_give_nan():
    assert math.isnan(O.sample_angle2(1.0 + 41.0 * math.sqrt(0.04), 1.0, 0.04, 0.5))
    assert math.isnan(O.sample_angle2(float("nan"), 1.2, 0.04, 0.5))


@pytest.mark.slow
def test_step_propagation_matches_reflected_brownian_motion():
    # The 2D counterpart of the 3D step-level pin (Sec. 3, Details; eq. genericGF): after one
    # step of isolated pairs the propagated pairs' (R, cos theta) follow the planar reflected
    # Brownian paths that met the circle, the side of the rotation is even (E[sin theta] = 0),
    # and keeping the free end point's direction is rejected.  tau = 0.5 is beyond the
    # small-time expansion, so the radial functions are the exact ones.
    from .test_oracle_angle3 import _moment_z, _step_angles

    tau, R0 = 0.5, 1.2
    r, c = _reflected_paths(R0, tau, 300, 100000, 3)
    wins = ((1.0, 1.3), (1.3, 1.7))
    funcs = (lambda x: x, lambda x: 2.0 * x * x - 1.0)  # cos theta, cos 2 theta
    R, cs, sn = _step_angles(2, tau, R0, 12000, False, 5, exact2d=True)
    assert len(R) > 6000
    assert _moment_z(R, cs, r, c, wins, funcs) < 4.0
    assert abs(sn.mean()) < 4.0 * sn.std() / math.sqrt(len(sn))
    R, cs, _ = _step_angles(2, tau, R0, 12000, True, 5, exact2d=True)
    assert _moment_z(R, cs, r, c, wins, funcs) > 6.0
