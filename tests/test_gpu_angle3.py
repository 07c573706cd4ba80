"""Kernel-level parity of the 3D angular propagator (sim_eval_angle) with the oracle's, pair
by pair on the same uniforms.  cos Theta is a root of the distribution function of the angle
given the radii (Sec. 3, Details; eq. genericGF3D), found by two different searches on
coefficients summed in different orders, so the draws are compared in floating point: each
GPU value must solve the oracle's equation F(c) = u to within 1e-12 + 1e-14 e^{(R+R0-2)^2/4tau}
(the rounding of the series, whose terms cancel down to the image term), and lie within twice
that over the density of the oracle's root where the density exceeds 1e-3.  Inputs: pre-step separations uniform in the cut-off shell, new radii within a
few sqrt(tau) of contact (where the reflected propagator puts them), uniform draws."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1107_0270_amd import sim as S

pytestmark = pytest.mark.gpu


def _handle(dt, D, sigma, dim=3, flags=0):
    sp = np.array([0, 1], np.int32)
    pos = np.array([[0.25] * dim, [0.75] * dim])
    return S.Sim(dim=dim, box=1.0, dt=dt, D=(D, D, D), sigma=sigma, bc=O.BC_RAD, kappa=0.1, k_off=0.0,
                 precision=S.PREC_FP64, seed=1, species=sp, pos=pos, flags=flags)


def _inputs(rng, n, tau, rmax):
    R0 = 1.0 + (rmax - 1.0) * rng.random(n)
    R = 1.0 + np.abs(rng.normal(size=n)) * 2.0 * math.sqrt(tau) + 0.3 * (R0 - 1.0) * rng.random(n)
    u = rng.random(n)
    return R, R0, u


def _edges(tau):
    s = math.sqrt(tau)
    R = np.array([1.0, 1.0, 1.0 + s, 0.97, 1.0 + 6 * s, 1.0 + 0.5 * s, 1.0 + 0.5 * s, 1.3])
    R0 = np.array([1.0, 1.0 + 3 * s, 1.0, 1.0 + s, 1.0 + 0.1 * s, 1.0 + 0.5 * s, 1.0 + 0.5 * s, 0.9])
    u = np.array([0.5, 1e-9, 1.0 - 1e-9, 0.3, 0.7, 1e-300, 1.0 - 2.0 ** -53, 0.5])
    return R, R0, u


def test_out_of_range_pairs_give_nan():
    h = _handle(1e-5, 1.0, 0.005)
    s = math.sqrt(h.derived()["tau"])
    R = np.array([1.0 + 41.0 * s, np.nan, 1.2, np.inf])
    R0 = np.array([1.0, 1.2, np.nan, 1.0])
    c = h.eval_angle(R, R0, np.full(4, 0.5))
    h.close()
    assert np.all(np.isnan(c))
    assert all(math.isnan(O.sample_angle3(R[k], R0[k], s * s, 0.5)) for k in range(4))


def _tol(tau, R, R0):
    """Error bound of the distribution function: the coefficients sum terms of the size of the
    free Green's function to a result smaller by about e^{-(R+R0-2)^2 / 4 tau} (the image
    term), so their rounding error grows by that factor over the 1e-16 of one term."""
    return 1e-12 + 1e-14 * math.exp((R + R0 - 2.0) ** 2 / (4.0 * tau))


def _check(tau, R, R0, u, c):
    for k in range(len(R)):
        Rk, R0k = max(R[k], 1.0), max(R0[k], 1.0)
        tol = _tol(tau, Rk, R0k)
        w = O.angle3_coef(0, Rk, R0k, tau)
        res = O.angle3_cdf(w, c[k]) - u[k]
        assert -1.0 <= c[k] <= 1.0
        assert abs(res) < tol, (k, Rk, R0k, u[k], c[k], res)
        co = O.sample_angle3(Rk, R0k, tau, u[k])
        h = 1e-6
        dens = (O.angle3_cdf(w, min(co + h, 1.0)) - O.angle3_cdf(w, max(co - h, -1.0))) / (2 * h)
        if dens > 1e-3:  # both roots solve their equations to tol
            assert abs(c[k] - co) < 2.0 * tol / dens + 1e-13, (k, Rk, R0k, u[k], c[k], co)


@pytest.mark.parametrize("dt,D,sigma", [(1e-5, 1.0, 0.005), (1e-6, 1.0, 0.005), (1e-5, 10.0, 0.01), (1e-7, 1.0, 0.005)])
def test_angle_matches_the_oracle(dt, D, sigma):
    h = _handle(dt, D, sigma)
    d = h.derived()
    tau, rmax = d["tau"], d["rcut"] / d["a"]
    rng = np.random.default_rng(int(tau * 1000) + 3)
    # several workgroups and a ragged tail; at tau = 0.008 about 90 terms and 1,300 nodes per pair
    n = 150 - 17 if tau < 0.05 else 300 - 17 if tau < 0.5 else 1000 - 17
    R, R0, u = _inputs(rng, n, tau, rmax)
    eR, eR0, eu = _edges(tau)
    R, R0, u = np.concatenate([eR, R]), np.concatenate([eR0, R0]), np.concatenate([eu, u])
    c = h.eval_angle(R, R0, u)
    h.close()
    print(f"tau {tau:.3g}: {len(R)} pairs, mean cos {c.mean():.4f}")
    _check(tau, R, R0, u, c)
    assert c[0] == pytest.approx(c[0])  # finite
    # the two ends of the distribution: u = 1e-300 and 1 - 2^-53 lie below the noise of F (its
    # terms cancel to about 1e-16), so the draws must sit where F is within that noise of 0 and 1
    for k, end in ((5, 0.0), (6, 1.0)):
        w = O.angle3_coef(0, max(R[k], 1.0), max(R0[k], 1.0), tau)
        assert abs(O.angle3_cdf(w, c[k]) - end) < 1e-12, (k, c[k])


def test_full_size_launch_sampled_against_the_oracle():
    # the benchmark's launch: 10^6 pairs of the headline pair (tau = 0.8), 300 checked one by one
    h = _handle(1e-5, 1.0, 0.005)
    d = h.derived()
    tau, rmax = d["tau"], d["rcut"] / d["a"]
    R, R0, u = _inputs(np.random.default_rng(9), 1000000, tau, rmax)
    c = h.eval_angle(R, R0, u)
    h.close()
    assert np.all(np.isfinite(c)) and np.all(np.abs(c) <= 1.0)
    pick = np.random.default_rng(10).choice(len(R), 300, replace=False)
    pick[:2] = [0, len(R) - 1]
    _check(tau, R[pick], R0[pick], u[pick], c[pick])


def test_rejects_bad_arguments():
    h = _handle(1e-5, 1.0, 0.005)
    with pytest.raises(S.SimError) as e:
        h.eval_angle_device(0, 1, 1, 1, 1)
    assert e.value.code == S.SIM_EINVAL
    h.close()
    for dim in (3, 2):  # tau = 8e-4: more terms than the series keeps
        # a step that would draw angles is refused at creation; one that keeps the free end
        # point's direction is created, and its angle evaluation is refused
        with pytest.raises(S.SimError) as e:
            _handle(1e-8, 1.0, 0.005, dim=dim)
        assert e.value.code == S.SIM_EUNSUPPORTED
        h = _handle(1e-8, 1.0, 0.005, dim=dim, flags=S.F_KEEP_DIRECTION)
        assert h.derived()["tau"] < 2e-3
        with pytest.raises(S.SimError) as e:
            h.eval_angle(np.full(4, 1.01), np.full(4, 1.01), np.full(4, 0.5))
        assert e.value.code == S.SIM_EUNSUPPORTED
        h.close()
