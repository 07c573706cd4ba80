"""Pins of the oracle's 3D angular propagator (CPU only).

After a non-reactive encounter the pair's new separation is drawn from G_ref - G_abs
(Sec. 2.2.2, eq. passage_prob): the radius from the radial propagator, then the angle
Theta to the old separation from J (G_ref - G_abs), J = 2 pi sin(Theta) r^2 (Sec. 3,
Details), with the Legendre series of eq. genericGF3D for the reflecting (h -> 0) and
absorbing (h -> infinity) surfaces.  The pins:
  - the half-integer Bessel functions against scipy's;
  - the n = 0 coefficient against the closed forms of Sec. 4.1 (w_0 = 4 pi sqrt(R R0)
    (g_ref - g_abs)), which fixes the quadrature and the boundary functions F_{1/2};
  - the same Bessel functions and rule on the free Green's function against Weber's
    integral, int e^{-tau x^2} J_nu(Rx) J_nu(R0x) x dx = e^{-(R^2+R0^2)/4tau} I_nu(R R0/2tau)
    / (2 tau), for every order;
  - the locally flat surface (tau -> 0, the pair a few sqrt(tau) from contact): the
    lateral displacement of the reflected part is Gaussian, variance 2 tau per coordinate,
    so P(Theta > theta) -> e^{-theta^2 R R0 / 4 tau} at the geometric-mean radius;
  - a Monte Carlo of reflected Brownian motion with fine sub-steps at tau = 0.5, whose
    encountered paths give the angular moments E[P_n(cos Theta) | R in a window];
  - the distribution function runs from 0 to 1, is monotone, and the draw inverts it.
"""
import math

import numpy as np
import pytest
from scipy import special as sp

import oracle as O


@pytest.mark.parametrize("z", [1e-3, 0.05, 0.7, 5.0, 40.0, 300.0])
def test_half_integer_bessel_functions(z):
    kmax = 161
    J, Y = O.bessel_half(kmax, z)
    nu = np.arange(kmax + 1) - 0.5
    Jr, Yr = sp.jv(nu, z), sp.yv(nu, z)
    scale = math.sqrt(2.0 / (math.pi * z))  # the envelope of both beyond the turning point
    ok = np.abs(Jr) > 1e-280
    tol = 1e-13 if z < 100 else 5e-11  # scipy's own accuracy at large arguments
    assert np.all(np.abs(J[ok] - Jr[ok]) <= tol * np.maximum(np.abs(Jr[ok]), 1e-6 * scale))
    ok = np.abs(Yr) < 1e300
    assert np.all(np.abs(Y[ok] - Yr[ok]) <= 2e-12 * np.maximum(np.abs(Yr[ok]), 1e-6 * scale))


CASES = [(1.5, 1.2, 0.8), (1.05, 1.0, 0.08), (2.2, 1.4, 0.8), (1.3, 1.25, 0.02), (1.0, 1.6, 0.3)]


@pytest.mark.parametrize("R,R0,tau", CASES)
def test_zeroth_coefficient_is_the_radial_closed_form(R, R0, tau):
    w = O.angle3_coef(0, R, R0, tau)
    L = O.lib()
    want = 4.0 * math.pi * math.sqrt(R * R0) * (L.orc_g3_rad(R, R0, tau, 0.0) - L.orc_g3_abs(R, R0, tau))
    assert abs(w[0] - want) <= 1e-11 * want


@pytest.mark.parametrize("R,R0,tau", CASES)
def test_free_space_terms_match_webers_integral(R, R0, tau):
    w = O.angle3_coef(1, R, R0, tau)
    nu = np.arange(len(w)) + 0.5
    want = math.exp(-(R - R0) ** 2 / (4.0 * tau)) / (2.0 * tau) * sp.ive(nu, R * R0 / (2.0 * tau))
    assert np.all(np.abs(w - want) <= 1e-12 * want[0])


@pytest.mark.parametrize("a,b", [(0.5, 0.8), (0.0, 1.0), (1.0, 0.2)])
def test_locally_flat_surface_gives_a_gaussian_lateral_step(a, b):
    tau = 2e-3
    s = math.sqrt(tau)
    R0, R = 1.0 + a * s, 1.0 + b * s
    w = O.angle3_coef(0, R, R0, tau)
    for th in (0.5 * s, s, 2.0 * s, 3.0 * s):
        F = O.angle3_cdf(w, math.cos(th))  # P(Theta >= th)
        assert abs(F - math.exp(-th * th * R * R0 / (4.0 * tau))) < 0.012


def _reflected_paths(R0, tau, M, npath, seed):
    """End radius and cos Theta of the paths that met the sphere: sub-steps of variance
    2 tau / M per coordinate, mirrored across the surface when they end inside it, and a
    contact in between detected with the flat-surface bridge probability."""
    rng = np.random.default_rng(seed)
    x = np.zeros((npath, 3))
    x[:, 0] = R0
    r = np.full(npath, R0)
    hit = np.zeros(npath, bool)
    dt = tau / M
    for _ in range(M):
        y = x + math.sqrt(2.0 * dt) * rng.standard_normal((npath, 3))
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
    r, c = _reflected_paths(R0, tau, 300, 100000, 11)
    xg, wg = np.polynomial.legendre.leggauss(12)
    for lo, hi in ((1.0, 1.3), (1.3, 1.7)):
        sel = (r >= lo) & (r < hi)
        n = sel.sum()
        Rs = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
        W = np.array([O.angle3_coef(0, Rv, R0, tau, 4) for Rv in Rs])
        # the radial weight of the window is r^2 x (angular integral) ~ R^{3/2} w_0
        m = (wg[:, None] * Rs[:, None] ** 1.5 * W).sum(0)
        for k, Pk in ((1, c[sel]), (2, 1.5 * c[sel] ** 2 - 0.5)):
            err = Pk.std() / math.sqrt(n)
            assert abs(Pk.mean() - m[k] / m[0]) < 4.0 * err + 0.006, (lo, k, Pk.mean(), m[k] / m[0])


@pytest.mark.parametrize("R,R0,tau", CASES)
def test_distribution_function_and_its_inverse(R, R0, tau):
    w = O.angle3_coef(0, R, R0, tau)
    cs = np.linspace(-1.0, 1.0, 801)
    F = np.array([O.angle3_cdf(w, c) for c in cs])
    assert abs(F[0]) < 1e-15 and abs(F[-1] - 1.0) < 1e-12
    assert np.min(np.diff(F)) > -1e-12
    for u in (1e-6, 0.2, 0.5, 0.93, 1.0 - 1e-9):
        c = O.sample_angle3(R, R0, tau, u)
        assert -1.0 <= c <= 1.0
        assert abs(O.angle3_cdf(w, c) - u) < 1e-12


def test_terms_follow_the_angular_spread():
    assert O.angle3_terms(1.0, 1.0, 0.8) == 8 + math.ceil(math.sqrt(45.0 / 0.8))
    assert O.angle3_terms(1.0, 1.0, 1e-4) == 160  # the cap
    w = O.angle3_coef(0, 1.4, 1.1, 0.08)
    assert abs(w[-1] / w[0]) < 1e-15  # the last term kept is negligible


def _step_angles(dim, tau, R0, M, keep_direction, seed, **kw):
    """One oracle step of M isolated pairs at separation R0 a (random orientations), reflecting
    surface: the new radius and the cosine (and in 2D the sine) of the angle between each
    propagated pair's separations before and after, from the positions."""
    from .test_oracle_sim import _isolated_pairs

    a, Deff = 0.005, 2.0
    sp, pos, box = _isolated_pairs(M, 0.25, R0 * a, dim, seed=seed)
    s = O.OracleSim(dim=dim, bc=O.BC_REF, box=[box] * dim, dt=tau * a * a / Deff, D=(1.0, 1.0, 0.5), sigma=a,
                    eps_cut=1e-14, species=sp, pos=pos, seed=seed, keep_direction=keep_direction, **kw)
    s.step()
    _, x, _ = s.state()
    mt = s.matches()
    i, j = mt["i"].astype(np.int64), mt["j"].astype(np.int64)
    mi = lambda d: d - box * np.round(d / box)
    r0v, rn = mi(pos[j] - pos[i]), mi(x[j] - x[i])
    n0, n1 = np.linalg.norm(r0v, axis=1), np.linalg.norm(rn, axis=1)
    cs = (r0v * rn).sum(1) / (n0 * n1)
    sn = (r0v[:, 0] * rn[:, 1] - r0v[:, 1] * rn[:, 0]) / (n0 * n1) if dim == 2 else None
    R = n1 / a
    assert np.abs(R - mt["Rpp"]).max() < 1e-9  # the placement has the drawn radius
    if not keep_direction:
        assert np.abs(cs - mt["cos_theta"]).max() < 1e-9  # and the drawn angle
    return R, cs, sn


def _moment_z(R, cs, r, c, windows, funcs):
    """Largest |difference| of window moments between the step and the Monte Carlo, in
    standard errors after a 0.006 allowance for the Monte Carlo's discretisation."""
    zs = []
    for lo, hi in windows:
        sa, sb = (R >= lo) & (R < hi), (r >= lo) & (r < hi)
        for f in funcs:
            A, B = f(cs[sa]), f(c[sb])
            d = max(abs(A.mean() - B.mean()) - 0.006, 0.0)
            zs.append(d / math.sqrt(A.var() / len(A) + B.var() / len(B)))
    return max(zs)


@pytest.mark.slow
def test_step_propagation_matches_reflected_brownian_motion():
    # Step level (Sec. 3, Details): the matched pairs of one step, re-propagated from their
    # pre-step separation R0 with the radius from w_3 r^2 (g_ref - g_abs) and the angle from
    # J (G_ref - G_abs), end where reflected Brownian paths that met the sphere end: their
    # (R, cos Theta) law is the normalised G_ref - G_abs.  The window moments E[P_1], E[P_2] of
    # cos Theta agree with the Monte Carlo; keeping the free end point's direction (the
    # reading this step replaced) does not.
    tau, R0 = 0.5, 1.2
    r, c = _reflected_paths(R0, tau, 300, 100000, 11)
    wins = ((1.0, 1.3), (1.3, 1.7))
    funcs = (lambda x: x, lambda x: 1.5 * x * x - 0.5)
    R, cs, _ = _step_angles(3, tau, R0, 40000, False, 3)
    assert len(R) > 20000
    assert _moment_z(R, cs, r, c, wins, funcs) < 4.0
    R, cs, _ = _step_angles(3, tau, R0, 40000, True, 3)
    assert _moment_z(R, cs, r, c, wins, funcs) > 6.0
