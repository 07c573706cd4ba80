"""Kernel-level parity of the 2D angular propagator (sim_eval_angle on a 2D handle) with the
oracle's, pair by pair on the same uniforms.  |theta| is a root of the distribution function of
the angle given the radii (Sec. 3, Details; eqs. genericGF, fRad), found by two different
searches on coefficients summed in different orders, so the draws are compared in floating
point: each GPU value must solve the oracle's equation F(t) = u to within
1e-12 + 1e-14 e^{(R+R0-2)^2/4tau} (the rounding of a series whose terms cancel down to the
image term), and lie within twice that over the density of the oracle's root where the density
exceeds 1e-3.  Inputs: membrane pairs with pre-step separations in the cut-off ring and new
radii within a few sqrt(tau) of contact."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1107_0270_amd import sim as S

pytestmark = pytest.mark.gpu


def _handle(dt, D, sigma):
    # the angular sampler does not use the small-time expansion, so handles beyond the tau at
    # which the expansion holds are accepted for it
    sp = np.array([0, 1], np.int32)
    pos = np.array([[0.25, 0.25], [0.75, 0.75]])
    return S.Sim(dim=2, box=1.0, dt=dt, D=(D, D, D), sigma=sigma, bc=O.BC_RAD, kappa=0.05, k_off=0.0,
                 precision=S.PREC_FP64, seed=1, species=sp, pos=pos, flags=S.F_UNVALIDATED_TAU)


def _tol(tau, R, R0):
    return 1e-12 + 1e-14 * math.exp((R + R0 - 2.0) ** 2 / (4.0 * tau))


def _check(tau, R, R0, u, th):
    for k in range(len(R)):
        Rk, R0k = max(R[k], 1.0), max(R0[k], 1.0)
        tol = _tol(tau, Rk, R0k)
        w = O.angle2_coef(0, Rk, R0k, tau)
        res = O.angle2_cdf(w, th[k]) - u[k]
        assert 0.0 <= th[k] <= math.pi
        assert abs(res) < tol, (k, Rk, R0k, u[k], th[k], res)
        to = O.sample_angle2(Rk, R0k, tau, u[k])
        h = 1e-6
        dens = (O.angle2_cdf(w, min(to + h, math.pi)) - O.angle2_cdf(w, max(to - h, 0.0))) / (2 * h)
        if dens > 1e-3:
            assert abs(th[k] - to) < 2.0 * tol / dens + 1e-13, (k, Rk, R0k, u[k], th[k], to)


# the membrane pair (D_eff = 0.2 um^2/s, a = 5 nm) at dt = 5 us and 1 us: tau = 0.04, 0.008;
# and D = 1 at dt = 5 us: tau = 0.2
@pytest.mark.parametrize("dt,D", [(5e-6, 0.1), (1e-6, 0.1), (5e-6, 0.5)])
def test_2d_angle_matches_the_oracle(dt, D):
    h = _handle(dt, D, 0.005)
    d = h.derived()
    tau, rmax = d["tau"], d["rcut"] / d["a"]
    rng = np.random.default_rng(int(tau * 1e4) + 5)
    n = 150 - 13 if tau < 0.01 else 300 - 13
    R0 = 1.0 + (rmax - 1.0) * rng.random(n)
    R = 1.0 + np.abs(rng.normal(size=n)) * 2.0 * math.sqrt(tau) + 0.3 * (R0 - 1.0) * rng.random(n)
    u = rng.random(n)
    s = math.sqrt(tau)
    eR = np.array([1.0, 1.0, 1.0 + s, 0.97, 1.0 + 6 * s, 1.0 + 0.5 * s, 1.0 + 0.5 * s])
    eR0 = np.array([1.0, 1.0 + 3 * s, 1.0, 1.0 + s, 1.0 + 0.1 * s, 1.0 + 0.5 * s, 1.0 + 0.5 * s])
    eu = np.array([0.5, 1e-9, 1.0 - 1e-9, 0.3, 0.7, 1e-300, 1.0 - 2.0 ** -53])
    R, R0, u = np.concatenate([eR, R]), np.concatenate([eR0, R0]), np.concatenate([eu, u])
    th = h.eval_angle(R, R0, u)
    h.close()
    print(f"2D tau {tau:.3g}: {len(R)} pairs, mean |theta| {th.mean():.4f}")
    _check(tau, R, R0, u, th)
    assert th[5] < 1e-3  # the lower end; at the upper end F reaches 1 - 2^-53 before pi (checked above)


def test_2d_large_launch_sampled_against_the_oracle():
    # 2 x 10^5 membrane pairs at tau = 0.04, 100 checked one by one
    h = _handle(5e-6, 0.1, 0.005)
    d = h.derived()
    tau, rmax = d["tau"], d["rcut"] / d["a"]
    rng = np.random.default_rng(12)
    n = 200000
    R0 = 1.0 + (rmax - 1.0) * rng.random(n)
    R = 1.0 + np.abs(rng.normal(size=n)) * 2.0 * math.sqrt(tau)
    u = rng.random(n)
    th = h.eval_angle(R, R0, u)
    h.close()
    assert np.all(np.isfinite(th)) and np.all((th >= 0.0) & (th <= math.pi))
    pick = np.random.default_rng(13).choice(n, 100, replace=False)
    pick[:2] = [0, n - 1]
    _check(tau, R[pick], R0[pick], u[pick], th[pick])


def test_2d_out_of_range_pairs_give_nan():
    h = _handle(5e-6, 0.1, 0.005)
    s = math.sqrt(h.derived()["tau"])
    th = h.eval_angle(np.array([1.0 + 41.0 * s, np.nan, 1.2]), np.array([1.0, 1.2, np.nan]), np.full(3, 0.5))
    h.close()
    assert np.all(np.isnan(th))
