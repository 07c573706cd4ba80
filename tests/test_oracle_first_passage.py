"""Pins of the oracle's first-passage bisection (the paper's Appendix), CPU only.

On the half line (eq. bayes1D) the bisection, with its midpoints and choices
conditioned on the encounter known to lie in the interval, locates the first
contact exactly in law.  The conditional density of the first-passage time s
of a bridge from x_i to x_f over T (distances beyond contact, time in units of
a^2 / D_eff, variance 2t per unit time) is
    f(s) = j(s | x_i) g(x_f, T - s | 0) / g(x_f, T | -x_i),
with j(s | x) = x / sqrt(4 pi s^3) e^{-x^2/4s} the first-passage density and g the
free Gaussian: the image term in the denominator is g_free - g_abs.  The tests
compare the located intervals with the bin probabilities of that law, check the
3D and 2D forms against it where the contact surface is locally flat (tau -> 0),
and check the exact special cases and invariants.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle as O

KEY = (2024, 11)


def _g(y, t, y0):
    return math.exp(-(y - y0) ** 2 / (4.0 * t)) / math.sqrt(4.0 * math.pi * t)


def _fpt_bins(xi, xf, T, nbins):
    """Probabilities of the bins [k, k + 1) * T / nbins of the conditional first-passage time."""
    norm = _g(xf, T, -xi)

    def f(s):
        if s <= 0.0 or s >= T:
            return 0.0
        return xi / math.sqrt(4.0 * math.pi * s ** 3) * math.exp(-xi * xi / (4.0 * s)) * _g(xf, T - s, 0.0) / norm

    edges = np.linspace(0.0, T, nbins + 1)
    pr = np.array([integrate.quad(f, edges[k], edges[k + 1], limit=200, epsabs=1e-13, epsrel=1e-11)[0]
                   for k in range(nbins)])
    return pr


def _chi2_pvalue(counts, probs):
    """Chi-square goodness of fit, adjacent bins merged until each expects >= 5 counts."""
    n = counts.sum()
    exp = probs * n
    obs_m, exp_m, co, ce = [], [], 0.0, 0.0
    for o, e in zip(counts, exp):
        co += o
        ce += e
        if ce >= 5.0:
            obs_m.append(co)
            exp_m.append(ce)
            co, ce = 0.0, 0.0
    if ce > 0:
        obs_m[-1] += co
        exp_m[-1] += ce
    obs_m, exp_m = np.array(obs_m), np.array(exp_m)
    chi2 = ((obs_m - exp_m) ** 2 / exp_m).sum()
    return stats.chi2.sf(chi2, len(obs_m) - 1)


def _sample(dim, xi, xf, tau, levels, m, step=0, n_terms=12):
    lo = np.empty(m, np.int64)
    att = np.empty(m, np.int64)
    for c in range(m):
        lo[c], att[c] = O.first_passage(dim, xi, xf, tau, levels, c, step, KEY, n_terms=n_terms)
    return lo, att


# (x_i, x_f, T): encounter probabilities e^{-x_i x_f / T} of 0.62, 0.05, 1 (ends at contact), 0.9
CASES_1D = [(0.6, 0.8, 1.0), (1.2, 1.0, 0.4), (0.7, 0.0, 0.5), (0.05, 0.4, 0.2)]


@pytest.mark.parametrize("xi,xf,T", CASES_1D)
def test_half_line_bisection_matches_the_first_passage_law(xi, xf, T):
    levels, nb = 6, 64
    lo, att = _sample(1, [1.0 + xi], [1.0 + xf], T, levels, 20000)
    assert lo.min() >= 0 and lo.max() < nb
    assert att.min() >= levels
    counts = np.bincount(lo, minlength=nb).astype(float)
    p = _fpt_bins(xi, xf, T, nb)
    assert abs(p.sum() - 1.0) < 1e-7  # the law is normalised: the image term is the encounter mass
    assert _chi2_pvalue(counts, p) > 1e-4


def test_unconditioned_choice_would_fail_the_pin():
    # the paper's steps read without the conditioning put the first contact in the
    # first half with probability P(s < T/2 | x_i, x_f), not P(s < T/2 | ..., encounter):
    # with an encounter probability of 0.62 the two differ by far more than the noise
    xi, xf, T = 0.6, 0.8, 1.0
    p = _fpt_bins(xi, xf, T, 2)
    p_enc = math.exp(-xi * xf / T)
    lo, _ = _sample(1, [1.0 + xi], [1.0 + xf], T, 1, 20000)
    frac = np.mean(lo == 0)
    assert abs(frac - p[0]) < 5 * math.sqrt(p[0] * (1 - p[0]) / 20000)
    assert abs(frac - p[0] * p_enc) > 20 * math.sqrt(p[0] * (1 - p[0]) / 20000)


@pytest.mark.parametrize("dim", [3, 2])
def test_locally_flat_contact_reduces_to_the_half_line(dim):
    # tau -> 0 with the pair a few sqrt(tau) from contact: the contact surface is flat on
    # the scale of the motion and the radial encounter probability tends to eq. bayes1D
    tau = 1e-6
    s = math.sqrt(tau)
    xi, xf = 0.6 * s, 0.8 * s
    e = np.zeros(dim)
    e[0] = 1.0
    levels, nb = 5, 32
    lo, _ = _sample(dim, (1.0 + xi) * e, (1.0 + xf) * e, tau, levels, 20000)
    counts = np.bincount(lo, minlength=nb).astype(float)
    p = _fpt_bins(xi, xf, tau, nb)
    assert _chi2_pvalue(counts, p) > 1e-4


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_start_at_contact_gives_the_first_interval(dim):
    # p1 = 1 at every level: the first contact is at the start
    xi = np.zeros(dim)
    xi[0] = 1.0
    xf = np.full(dim, 1.3)
    for c in range(50):
        lo, att = O.first_passage(dim, xi, xf, 0.3, 12, c, 5, KEY)
        assert lo == 0 and att == 12


def test_draws_are_keyed():
    a = O.first_passage(3, [1.2, 0.1, 0.0], [0.9, 0.8, 0.1], 0.4, 16, 7, 3, KEY)
    assert a == O.first_passage(3, [1.2, 0.1, 0.0], [0.9, 0.8, 0.1], 0.4, 16, 7, 3, KEY)
    others = {O.first_passage(3, [1.2, 0.1, 0.0], [0.9, 0.8, 0.1], 0.4, 16, c, 3, KEY)[0] for c in range(20)}
    assert len(others) > 10


def test_deeper_levels_refine_the_same_interval():
    # level l + 1 draws nothing new for levels <= l: its interval lies inside level l's
    for c in range(30):
        lo8, _ = O.first_passage(3, [1.1, 0.2, 0.0], [1.0, 0.6, 0.2], 0.5, 8, c, 1, KEY)
        lo12, _ = O.first_passage(3, [1.1, 0.2, 0.0], [1.0, 0.6, 0.2], 0.5, 12, c, 1, KEY)
        assert lo12 >> 4 == lo8


def test_exhausted_level_ends_the_refinement():
    # an interval with no realistic encounter (p_enc ~ e^-841): every proposal of the first
    # level is rejected; the refinement stops there with the flag set
    lo, att = O.first_passage(3, [3.9, 0.0, 0.0], [3.9, 0.0, 0.0], 0.01, 10, 0, 0, KEY)
    assert lo == 0 and att == (4096 | 0x80000000)
    # a pair that exhausts a later level keeps the interval it reached, at the full resolution
    for c in range(200):
        lo, att = O.first_passage(1, [1.0 + 0.02], [1.0 + 0.02], 1e-3, 16, c, 0, KEY)
        assert att & 0x80000000 == 0 or lo % 2 == 0
