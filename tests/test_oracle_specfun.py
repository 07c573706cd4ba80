"""Pins of the oracle's generator and special functions (CPU only).

Each function is checked against something other than itself: published
known-answer vectors, SciPy's implementations, or 40-digit mpmath evaluations of
the defining integrals.
"""
import math
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import special as S

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert O.philox(ctr, key) == out


def test_u01_open_interval():
    assert O.u01(0) == 0.5 * 2.0 ** -32
    assert O.u01(0xFFFFFFFF) == 1.0 - 0.5 * 2.0 ** -32
    assert 0.0 < O.u01(0) < O.u01(1) < 1.0


@pytest.mark.parametrize("x", [0.0, 1e-8, 0.3, 1.0, 2.5, 2.999, 3.0, 3.001, 4.0, 7.5, 20.0, 1e3, 1e6])
def test_erfcx_vs_scipy(x):
    assert O.erfcx(x) == pytest.approx(S.erfcx(x), rel=2e-15, abs=0)


@pytest.mark.parametrize("x", [0.0, 0.01, 1.0, 5.0, 12.0, 19.99, 20.0, 20.01, 35.0, 300.0, 1e5])
def test_i0e_vs_scipy(x):
    assert O.i0e(x) == pytest.approx(S.i0e(x), rel=4e-15, abs=0)


def _ierfcx_exact(n, x):
    """e^{x^2} i^n erfc(x) = (2/sqrt(pi)) int_0^inf u^n/n! e^{-u^2 - 2xu} du (Cauchy form of eq. iErf)."""
    mp.mp.dps = 40
    x = mp.mpf(x)
    if n == -1:
        return 2 / mp.sqrt(mp.pi)
    f = lambda u: u ** n / mp.factorial(n) * mp.exp(-u * u - 2 * x * u)
    return 2 / mp.sqrt(mp.pi) * mp.quad(f, [0, 1, 5, mp.inf])


@pytest.mark.parametrize("x", [0.0, 0.25, 1.0, 2.0, 5.0])
def test_ierfcx_vs_integral(x):
    kmax = 16
    got = O.ierfcx(x, kmax)
    for k in range(-1, kmax + 1):
        ref = float(_ierfcx_exact(k, x))
        # the upward recursion is exact up to rounding growth; what enters the
        # expansions is i^{k-1} times (2 sqrt tau)^k, so compare on the scale of
        # the k = 0 value
        assert abs(got[k + 1] - ref) <= 1e-13 * abs(ref) + 1e-14 * got[1], (k, x)


def test_ierfc_special_values():
    # i^1 erfc closed form (Sec. 4.2) and i^n erfc(0) = 1 / (2^n Gamma(1 + n/2))
    for x in [0.1, 0.7, 2.3]:
        v = O.ierfcx(x, 3)
        assert v[2] * math.exp(-x * x) == pytest.approx(math.exp(-x * x) / math.sqrt(math.pi) - x * math.erfc(x), rel=1e-13)
    v = O.ierfcx(0.0, 12)
    for n in range(0, 13):
        assert v[n + 1] == pytest.approx(1.0 / (2.0 ** n * math.gamma(1 + n / 2)), rel=1e-13)


def test_asym_coeffs_closed_form():
    # a_k(nu) of eq. coeffDef against the product written out by hand for k <= 3
    for nu in [0.0, 1.0, 0.5, 2.0]:
        m = 4 * nu * nu
        a = O.asym_coeffs(nu, 3)
        assert a[0] == 1.0
        assert a[1] == pytest.approx((m - 1) / 8)
        assert a[2] == pytest.approx((m - 1) * (m - 9) / (2 * 64))
        assert a[3] == pytest.approx((m - 1) * (m - 9) * (m - 25) / (6 * 512))
    # half-integer order terminates: K_{1/2} is elementary (Sec. 4.1), a_k(1/2) = 0 for k >= 1
    assert np.all(O.asym_coeffs(0.5, 6)[1:] == 0.0)


def test_asym_series_reproduces_bessel():
    # the expansions of I_0, K_0, I_1, K_1 quoted in Sec. 4.2, truncated at a
    # few terms, against SciPy at large argument
    x = 40.0
    for nu in [0, 1]:
        a = O.asym_coeffs(nu, 8)
        k = np.arange(9)
        ival = math.exp(x) / math.sqrt(2 * math.pi * x) * np.sum((-1.0) ** k * a / x ** k)
        kval = math.sqrt(math.pi / (2 * x)) * math.exp(-x) * np.sum(a / x ** k)
        assert ival == pytest.approx(S.iv(nu, x), rel=1e-12)
        assert kval == pytest.approx(S.kv(nu, x), rel=1e-12)


@pytest.mark.parametrize("yc", [0.0, 0.3, 1.7, 6.0, 25.0])
@pytest.mark.parametrize("u", [1e-300, 1e-12, 0.01, 0.5, 0.999999])
def test_erfc_tail_inverse(yc, u):
    y = O.erfc_tail_inv(yc, u)
    assert y >= yc
    mp.mp.dps = 40
    lhs = mp.log(mp.erfc(mp.mpf(y)))
    rhs = mp.log(mp.mpf(u)) + mp.log(mp.erfc(mp.mpf(yc)))
    assert float(lhs - rhs) == pytest.approx(0.0, abs=1e-12 * max(1.0, abs(float(rhs))))
