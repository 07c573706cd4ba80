"""Kernel-level parity of the pair probabilities: p_enc and p_reac from the step's own device
functions (sim_eval_pairs) against the oracle, element by element, over (R, R0) points that
cover the pair domain within r_cut.  Tolerances as in the trajectory parity tests: p_enc 1e-12
(binary64, 3D), 1e-11 (binary64 2D expansion), 1e-6 (binary32 exponentials of binary64
arguments), 1e-4 (plain binary32); p_reac (binary64 in every mode) 1e-9."""
import numpy as np
import pytest

import oracle as O
from paper_1107_0270_amd import sim as S

pytestmark = pytest.mark.gpu


def _handle(dim, bc, prec, dt, D, sigma, kappa, n_terms=12):
    sp = np.array([0, 1], np.int32)
    pos = np.array([[0.25] * dim, [0.75] * dim])
    return S.Sim(dim=dim, box=1.0, dt=dt, D=D, sigma=sigma, bc=bc, kappa=kappa, k_off=0.0, precision=prec,
                 n_terms=n_terms, species=sp, pos=pos)


def _points(rng, n, rmax, spread):
    R = 1.0 + (rmax - 1.0) * rng.random(n)
    R0 = 1.0 + (rmax + spread - 1.0) * rng.random(n)
    R[:8] = [1.0 + 1e-9, 1.0 + 1e-6, 1.001, 1.01, rmax, 1.5, 2.0, 3.0]
    R0[:8] = [1.0, 1.0, 1.0 + 1e-7, 1.002, rmax, 1.0, 1.5, 3.0]
    return R, R0


CASES_3D = [  # (bc, precision, kappa, dt, p_enc tolerance)
    (O.BC_RAD, S.PREC_FP64, 0.1, 1e-5, 1e-12),
    (O.BC_RAD, S.PREC_FP32_FP64NC, 0.1, 1e-5, 1e-6),
    (O.BC_RAD, S.PREC_FP32, 0.1, 1e-5, 1e-4),
    (O.BC_RAD, S.PREC_FP64, 1.0, 1e-6, 1e-12),
    (O.BC_ABS, S.PREC_FP64, 0.0, 1e-6, 1e-12),
    (O.BC_REF, S.PREC_FP32_FP64NC, 0.0, 1e-5, 1e-6),
]


@pytest.mark.parametrize("bc,prec,kappa,dt,tol", CASES_3D)
def test_pair_probabilities_3d(bc, prec, kappa, dt, tol):
    sigma, D = 0.005, (1.0, 1.0, 0.5)
    h = _handle(3, bc, prec, dt, D, sigma, kappa)
    der = h.derived()
    tau, hh, rmax = der["tau"], der["hh"], der["rcut"] / sigma
    rng = np.random.default_rng(42)
    R, R0 = _points(rng, 20000, rmax, 6.0 * np.sqrt(tau))
    pe, pr = h.eval_pairs(R, R0)
    oe = np.array([O.penc3(r, r0, tau) for r, r0 in zip(R, R0)])
    err = np.abs(pe - oe)
    print(f"tau {tau:.3g} h {hh:.3g}: max |dp_enc| {err.max():.2e}")
    assert err.max() <= tol
    if bc == O.BC_RAD:
        orr = np.array([O.preac3(r, r0, tau, hh) for r, r0 in zip(R, R0)])
        e2 = np.abs(pr - orr)
        print(f"  max |dp_reac| {e2.max():.2e}")
        assert e2.max() <= 1e-9
    else:
        assert np.all(pr == (1.0 if bc == O.BC_ABS else 0.0))
    # overlap rule
    po, _ = h.eval_pairs(np.array([0.5, 1.0]), np.array([1.0, 1.0]), preac=False)
    assert np.all(po == 1.0)


@pytest.mark.parametrize("prec,tol,n_terms", [(S.PREC_FP64, 1e-11, 12), (S.PREC_FP32_FP64NC, 1e-11, 12),
                                              (S.PREC_FP64, 1e-11, 10)])
def test_pair_probabilities_2d_small_tau(prec, tol, n_terms):
    # membrane workload at tau = 0.04 (dt = 5 us): the expansion is binary64 in every mode.
    # Order 12 runs the kernels compiled for it, order 10 the run-time-order form.
    sigma, D, kappa = 0.005, (0.1, 0.1, 0.05), 0.05
    h = _handle(2, O.BC_RAD, prec, 5e-6, D, sigma, kappa, n_terms=n_terms)
    der = h.derived()
    tau, hh, rmax = der["tau"], der["hh"], der["rcut"] / sigma
    rng = np.random.default_rng(7)
    R, R0 = _points(rng, 20000, rmax, 6.0 * np.sqrt(tau))
    pe, pr = h.eval_pairs(R, R0)
    oe = np.array([O.penc2(r, r0, tau, n_terms) for r, r0 in zip(R, R0)])
    orr = np.array([O.preac2(r, r0, tau, hh, n_terms) for r, r0 in zip(R, R0)])
    e1, e2 = np.abs(pe - oe), np.abs(pr - orr)
    print(f"tau {tau:.3g} h {hh:.3g}: max |dp_enc| {e1.max():.2e} max |dp_reac| {e2.max():.2e}")
    assert e1.max() <= tol
    assert e2.max() <= 1e-9


PROP_CASES = [  # (dim, dt, D, kappa, n_terms)
    (3, 1e-5, (1.0, 1.0, 0.5), 0.1, 12),   # tau = 0.8
    (3, 1e-6, (1.0, 1.0, 0.5), 0.1, 12),   # tau = 0.08
    (2, 5e-6, (0.1, 0.1, 0.05), 0.05, 12),  # tau = 0.04, compiled order
    (2, 5e-6, (0.1, 0.1, 0.05), 0.05, 10),  # run-time order
]


@pytest.mark.parametrize("wave", [True, False])
@pytest.mark.parametrize("dim,dt,D,kappa,n_terms", PROP_CASES)
def test_propagator_draws_match_the_oracle(dim, dt, D, kappa, n_terms, wave):
    # the step's rejection sampler, draw by draw, against the oracle's, on the same counters:
    # both forms (attempts over a wave, one draw per lane) must give the oracle's R'' and
    # attempt count
    seed, step = 11, 7
    sp = np.array([0, 1], np.int32)
    pos = np.array([[0.25] * dim, [0.75] * dim])
    h = S.Sim(dim=dim, box=1.0, dt=dt, D=D, sigma=0.005, bc=O.BC_RAD, kappa=kappa, k_off=0.0,
              precision=S.PREC_FP64, n_terms=n_terms, seed=seed, species=sp, pos=pos)
    tau = h.derived()["tau"]
    rng = np.random.default_rng(3)
    n = 4000
    R0 = 1.0 + 4.0 * rng.random(n) ** 2
    R0[:4] = [1.0, 1.0 + 1e-9, 2.0 / 0.5 + 1.0, 5.0]  # contact, near contact, past the mixture bound
    Rg, ag = h.eval_propagator(R0, step, wave=wave)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    ref = [O.sample_prop(dim, r0, tau, n_terms, (i, 0xFFFFFFFF, step, 5), key) for i, r0 in enumerate(R0)]
    Ro = np.array([r[0] for r in ref])
    ao = np.array([r[1] for r in ref])
    bad = np.flatnonzero(ag != ao)
    print(f"dim {dim} tau {tau:.3g} n {n_terms} wave {wave}: attempts differ at {len(bad)}; "
          f"max |dR''| {np.abs(Rg - Ro).max():.2e}")
    assert len(bad) == 0, (bad[:5], R0[bad[:5]], ag[bad[:5]], ao[bad[:5]])
    assert np.abs(Rg - Ro).max() <= 1e-9
