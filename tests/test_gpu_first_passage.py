"""Kernel-level parity of the first-passage bisection (sim_eval_first_passage, the paper's
Appendix) against the oracle's, pair by pair on the same counters, in 3D and 2D.  The located interval is an
integer and the attempt count too, so both must agree exactly; the decisions behind them are
taken in binary64 on both sides.  Inputs are the step's candidates: a pre-step separation
uniform in the shell 1 < R0 < r_cut / a, a free step of sqrt(2 tau) per coordinate, kept with
the oracle's encounter probability."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1107_0270_amd import sim as S

pytestmark = pytest.mark.gpu


def _handle(dt, D, sigma, seed, dim=3, **kw):
    sp = np.array([0, 1], np.int32)
    pos = np.array([[0.25] * dim, [0.75] * dim])
    return S.Sim(dim=dim, box=1.0, dt=dt, D=(D, D, D), sigma=sigma, bc=O.BC_RAD, kappa=0.1 if dim == 3 else 0.05,
                 k_off=0.0, precision=S.PREC_FP64, seed=seed, species=sp, pos=pos, **kw)


def _penc(dim, R, R0, tau):
    return O.penc3(R, R0, tau) if dim == 3 else O.penc2(R, R0, tau, 12)


def _candidates(rng, n, tau, rmax, dim=3):
    """Separation vectors (n, 3) before and after the step; 2D pairs have a zero third component."""
    out_i, out_f = [], []
    while sum(len(x) for x in out_i) < n:
        m = 4 * n
        d = rng.normal(size=(m, dim))
        d /= np.linalg.norm(d, axis=1)[:, None]
        R0 = (1.0 + (rmax ** dim - 1.0) * rng.random(m)) ** (1.0 / dim)
        xi = d * R0[:, None]
        xf = xi + math.sqrt(2.0 * tau) * rng.normal(size=(m, dim))
        p = np.array([_penc(dim, np.linalg.norm(b), np.linalg.norm(a), tau) for a, b in zip(xi, xf)])
        keep = rng.random(m) < p
        out_i.append(xi[keep])
        out_f.append(xf[keep])
    xi, xf = np.concatenate(out_i)[:n], np.concatenate(out_f)[:n]
    if dim == 2:
        xi, xf = np.pad(xi, ((0, 0), (0, 1))), np.pad(xf, ((0, 0), (0, 1)))
    return xi, xf


def _edge_pairs():
    # start at contact, end at contact, end overlapping, no motion, the far edge
    xi = np.array([[1.0, 0, 0], [1.3, 0.2, 0], [1.2, 0, 0], [1.1, 0.1, 0.1], [0, 1.0, 0]])
    xf = np.array([[1.4, 0.3, 0], [1.0, 0, 0], [0.7, 0.1, 0], [1.1, 0.1, 0.1], [0, 0, 1.0]])
    return xi, xf


CASES = [  # dt, D of each species (D_eff = 2D), sigma: tau = 0.08, 0.8 (the headline pair), 4
    (1e-6, 1.0, 0.005),
    (1e-5, 1.0, 0.005),
    (1e-5, 10.0, 0.01),
]


@pytest.mark.parametrize("levels", [1, 12, 40])
@pytest.mark.parametrize("dt,D,sigma", CASES)
def test_bisection_matches_the_oracle(dt, D, sigma, levels):
    seed, step = 17, 9
    h = _handle(dt, D, sigma, seed)
    d = h.derived()
    tau, rmax = d["tau"], d["rcut"] / d["a"]
    rng = np.random.default_rng(int(tau * 1000) + levels)
    xi, xf = _candidates(rng, 1500 - 37, tau, rmax)  # several workgroups and a ragged tail
    ei, ef = _edge_pairs()
    xi, xf = np.concatenate([ei, xi]), np.concatenate([ef, xf])
    lo, att = h.eval_first_passage(xi, xf, levels, step)
    h.close()
    key = (seed & 0xFFFFFFFF, seed >> 32)
    ref = [O.first_passage(3, xi[k], xf[k], tau, levels, k, step, key) for k in range(len(xi))]
    lo_o = np.array([r[0] for r in ref], np.uint64)
    att_o = np.array([r[1] for r in ref], np.uint32)
    bad = np.flatnonzero((lo != lo_o) | (att != att_o))
    print(f"tau {tau:.3g} levels {levels}: {len(xi)} pairs, mean attempts {att.mean():.2f}, {len(bad)} differ")
    assert len(bad) == 0, (bad[:5], lo[bad[:5]], lo_o[bad[:5]], att[bad[:5]], att_o[bad[:5]])
    assert lo[0] == 0  # contact at the start
    assert np.all(lo < (1 << levels)) and np.all(att >= levels)


@pytest.mark.parametrize("levels", [1, 12, 40])
@pytest.mark.parametrize("dt", [5e-6, 1e-6])
def test_2d_bisection_matches_the_oracle(dt, levels):
    # the membrane pair (D_eff = 0.2 um^2/s, a = 5 nm): tau = 0.04 and 0.008, expansion of order 12
    seed, step = 23, 4
    h = _handle(dt, 0.1, 0.005, seed, dim=2)
    d = h.derived()
    tau, rmax = d["tau"], d["rcut"] / d["a"]
    rng = np.random.default_rng(int(tau * 1e4) + levels)
    xi, xf = _candidates(rng, 1200 - 19, tau, rmax, dim=2)
    ei, ef = _edge_pairs()
    ei[:, 2] = 0.0
    ef[:, 2] = 0.0
    ei[4], ef[4] = [0, 1.0, 0], [1.0, 0, 0]
    xi, xf = np.concatenate([ei, xi]), np.concatenate([ef, xf])
    lo, att = h.eval_first_passage(xi, xf, levels, step)
    h.close()
    key = (seed & 0xFFFFFFFF, seed >> 32)
    ref = [O.first_passage(2, xi[k][:2], xf[k][:2], tau, levels, k, step, key) for k in range(len(xi))]
    lo_o = np.array([r[0] for r in ref], np.uint64)
    att_o = np.array([r[1] for r in ref], np.uint32)
    bad = np.flatnonzero((lo != lo_o) | (att != att_o))
    print(f"2D tau {tau:.3g} levels {levels}: {len(xi)} pairs, mean attempts {att.mean():.2f}, {len(bad)} differ")
    assert len(bad) == 0, (bad[:5], lo[bad[:5]], lo_o[bad[:5]], att[bad[:5]], att_o[bad[:5]])
    assert lo[0] == 0


def test_full_size_launch_sampled_against_the_oracle():
    # the benchmark's launch: 10^6 candidates of the headline pair at 20 levels, 400 of them
    # checked one by one
    seed, step, levels = 0, 1, 20
    h = _handle(1e-5, 1.0, 0.005, seed)
    d = h.derived()
    tau, rmax = d["tau"], d["rcut"] / d["a"]
    rng = np.random.default_rng(5)
    xi, xf = _candidates(rng, 20000, tau, rmax)
    reps = 50
    xi, xf = np.tile(xi, (reps, 1)), np.tile(xf, (reps, 1))  # 10^6 pairs (their own draws per index)
    lo, att = h.eval_first_passage(xi, xf, levels, step)
    h.close()
    key = (seed & 0xFFFFFFFF, seed >> 32)
    pick = np.random.default_rng(6).choice(len(xi), 400, replace=False)
    pick[:2] = [0, len(xi) - 1]
    for k in pick:
        lo_o, att_o = O.first_passage(3, xi[k], xf[k], tau, levels, int(k), step, key)
        assert (int(lo[k]), int(att[k])) == (lo_o, att_o), k


def test_rejects_bad_arguments_and_unsupported_2d_handles():
    h = _handle(1e-5, 1.0, 0.005, 0)
    xi, xf = _edge_pairs()
    for lv in (0, 53):
        with pytest.raises(S.SimError) as e:
            h.eval_first_passage(xi, xf, lv)
        assert e.value.code == S.SIM_EINVAL
    h.close()
    for kw in (dict(n_terms=10), dict(green2d=S.G2_EXACT)):  # only the order-12 expansion is built in 2D
        h2 = _handle(5e-6, 0.1, 0.005, 0, dim=2, **kw)
        with pytest.raises(S.SimError) as e:
            h2.eval_first_passage(xi, xf, 4)
        assert e.value.code == S.SIM_EUNSUPPORTED
        h2.close()
