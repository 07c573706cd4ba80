"""Exact 2D radial functions (sim_config.green2d = SIM_G2_EXACT) against the oracle's quadrature
of the same functions, beyond the small-time regime: element by element (p_enc, p_reac through
sim_eval_pairs), draw by draw (R'' through sim_eval_propagator) and step by step (the 2D membrane
workload as written, tau = 0.8).

Both sides use the exact functions for R0 up to 1 + 8.4 sqrt(tau) and the small-time expansions
beyond (the oracle's rule).  Tolerances, from the tables' bicubic interpolation (R steps of
sqrt(tau)/160, R0 steps of sqrt(tau)/40; the quadratures themselves agree to ~1e-12):
  * p_enc: 1e-6.
  * p_reac: 1e-6 where the boundary part exceeds 1e-4 of the free part.  p_reac is a ratio of
    boundary parts, and the quadrature's integrand oscillates with an amplitude up to ~1e5 times
    the result, so the two sides' Bessel functions (device library, C library), rounded
    differently, give noise of relative size ~1e-9 / (boundary / free) in p_reac.
  * R'': the device draws the exact distribution's quantile at a uniform within 1e-6 of its own
    (the oracle's distribution function at the device's R''), and R'' within 1e-6 of the
    oracle's inversion.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1107_0270_amd import sim as S

from .parity import make_pair, run

pytestmark = pytest.mark.gpu

MEM2D = dict(D=(0.1, 0.1, 0.05), sigma=0.005, kappa=0.05)


def _handle(dt, seed=0):
    sp = np.array([0, 1], np.int32)
    pos = np.array([[0.25, 0.25], [0.75, 0.75]])
    return S.Sim(dim=2, box=1.0, dt=dt, bc=O.BC_RAD, k_off=0.0, precision=S.PREC_FP64, seed=seed, species=sp, pos=pos,
                 green2d=S.G2_EXACT, **MEM2D)


@pytest.mark.parametrize("dt", [1e-4, 5e-6])  # tau = 0.8 (the workload as written) and 0.04
def test_exact_pair_probabilities(dt):
    h = _handle(dt)
    d = h.derived()
    tau, hh, Rc = d["tau"], d["hh"], d["rcut"] / d["a"]
    sw = O.x2_switch(tau)
    rng = np.random.default_rng(5)
    n = 400
    R = 1.0 + (Rc - 1.0) * rng.random(n)
    R0 = 1.0 + (sw + 2.0 * math.sqrt(tau) - 1.0) * rng.random(n)
    R[:8] = [1.0 + 1e-9, 1.0 + 1e-4, Rc, 1.3, 2.0, 1.01, 1.002, 1.0 + 1e-3]
    R0[:8] = [1.0, 1.2, 1.0, 1.0 + 1e-6, 2.0, 3.0, sw, sw + 1e-6]
    pe, pr = h.eval_pairs(R, R0)
    exact = R0 <= sw
    oe = np.array([O.penc2x(a, b, tau) if x else O.penc2(a, b, tau, 12) for a, b, x in zip(R, R0, exact)])
    orr = np.array([O.preac2x(a, b, tau, hh) if x else O.preac2(a, b, tau, hh, 12) for a, b, x in zip(R, R0, exact)])
    g = np.array([O.g2x(a, b, tau, hh) for a, b in zip(R, R0)])
    gf = np.array([O.g2_free(a, b, tau) for a, b in zip(R, R0)])
    cond = ((g[:, 1] - g[:, 0]) > 1e-4 * gf) | ~exact
    de, dr = np.abs(pe - oe), np.abs(pr - orr)[cond]
    far = (~exact).sum()
    print(f"tau {tau}: max |dp_enc| {de.max():.2e} (beyond the switch {de[~exact].max() if far else 0:.1e}), "
          f"max |dp_reac| {dr.max():.2e} over {cond.sum()} of {n}, {far} beyond the switch")
    idx = np.flatnonzero(cond)
    for k in idx[np.argsort(-np.abs(pr - orr)[cond])][:4]:
        print(f"  p_reac at R {R[k]:.6f} R0 {R0[k]:.6f}: device {pr[k]:.9f} oracle {orr[k]:.9f} "
              f"bc/free {(g[k, 1] - g[k, 0]) / gf[k]:.1e} exact {exact[k]}")
    assert far > 10
    assert de[exact].max() <= 1e-6 and dr.max() <= 1e-6
    assert de[~exact].max() <= 1e-9  # the same expansion on both sides
    h.close()


@pytest.mark.parametrize("wave", [True, False])
def test_exact_propagator_inverts_the_distribution_function(wave):
    seed, step = 13, 4
    h = _handle(1e-4, seed=seed)
    tau = h.derived()["tau"]
    sw = O.x2_prop_switch(tau)
    rng = np.random.default_rng(8)
    n = 200
    R0 = 1.0 + (sw - 1.0) * rng.random(n) ** 2
    R0[:5] = [1.0, 1.0 + 1e-8, sw, sw + 1e-6, sw + 1.0]
    Rg, att = h.eval_propagator(R0, step, wave=wave)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    errF, errR = 0.0, 0.0
    for i, r0 in enumerate(R0):
        if r0 > sw:  # beyond the switch: the rejection sampler on the expansions, draw for draw
            Ro, ao, _ = O.sample_prop(2, r0, tau, 12, (i, 0xFFFFFFFF, step, 5), key)
            assert att[i] == ao and abs(Rg[i] - Ro) <= 1e-9
            continue
        assert att[i] == 1
        u = O.u01(O.philox((i, 0xFFFFFFFF, step, 5), key)[0])
        top = r0 + 12 * math.sqrt(tau) + 1
        mt, m = O.m2x(top, r0, tau), O.m2x(Rg[i], r0, tau)
        errF = max(errF, abs((m[1] - m[0]) / (mt[1] - mt[0]) - u))
        # R'' against the oracle's own inversion, in probability: |dR''| times the density there.
        # At the switch the propagator's mass is about erfc(4.2) = 3e-9, which the two
        # quadratures resolve to a few 1e-7 of F, so R'' itself is no better than that over the
        # density (up to a few 1e-6 in R there).
        Ro = O.sample_prop2x(r0, tau, u)
        e = 1e-5
        dens = (O.m2x(Ro + e, r0, tau)[1] - O.m2x(Ro + e, r0, tau)[0] - O.m2x(Ro - e, r0, tau)[1]
                + O.m2x(Ro - e, r0, tau)[0]) / (2 * e * (mt[1] - mt[0]))
        errR = max(errR, abs(Rg[i] - Ro) * dens)
    print(f"wave {wave}: max |F(R'') - u| {errF:.2e}, max |dR''| x density {errR:.2e}")
    assert errF <= 1e-6 and errR <= 1e-6
    h.close()


def test_mem2d_as_written_exact_step_parity():
    # the 2D membrane workload as written (tau = 0.8, dt = 100 us) at its density (1,250 A and B
    # per um^2), 800 + 800 particles, binary64 state.  R'' comes from interpolated tables, so a
    # product may land within ~1e-9 um of the oracle's: positions are held to 1e-7 um in lock step.
    n = 800
    box = float(np.float32(math.sqrt(2 * n / 2500.0)))
    from paper_1107_0270_amd import inputs as I
    sp, pos, _ = I.uniform_state(n, n, box=box, dim=2, sigma=0.005, seed=21, f32=False)
    gpu, orc = make_pair(dim=2, bc=O.BC_RAD, box=box, dt=1e-4, k_off=2000.0, precision=S.PREC_FP64, species=sp,
                         pos=pos, seed=9, exact2d=True, **MEM2D)
    rep = run(gpu, orc, 6, p_tol=1e-6, pos_tol=1e-7, box=box, lockstep=True)
    print(rep)
    assert rep.pair_set_mismatch == 0 and rep.draw_mismatch == 0
    assert rep.unexplained == 0, rep.notes
    assert rep.max_dp <= 1e-6
    assert rep.max_dRpp <= 1e-4 and rep.max_dpreac <= 1e-6
    assert rep.near_decisions <= 2
    assert rep.reactions > 0 and rep.matches > 0


def test_exact_tables_at_large_intrinsic_rate():
    # h = 20 (kappa_2D = 2 pi D_eff h): the expansion's p_reac diverges there, the tables hold
    kw = dict(MEM2D)
    kw["kappa"] = 2 * math.pi * 0.2 * 20.0
    sp = np.array([0, 1], np.int32)
    pos = np.array([[0.25, 0.25], [0.75, 0.75]])
    h = S.Sim(dim=2, box=1.0, dt=5e-6, bc=O.BC_RAD, k_off=0.0, precision=S.PREC_FP64, species=sp, pos=pos,
              green2d=S.G2_EXACT, **kw)
    d = h.derived()
    tau, hh, Rc = d["tau"], d["hh"], d["rcut"] / d["a"]
    assert hh == pytest.approx(20.0)
    sw = O.x2_switch(tau)
    rng = np.random.default_rng(9)
    R = 1.0 + (Rc - 1.0) * rng.random(200)
    R0 = 1.0 + (sw - 1.0) * rng.random(200)
    _, pr = h.eval_pairs(R, R0)
    g = np.array([O.g2x(a, b, tau, hh) for a, b in zip(R, R0)])
    gf = np.array([O.g2_free(a, b, tau) for a, b in zip(R, R0)])
    cond = (g[:, 1] - g[:, 0]) > 1e-4 * gf
    orr = np.array([O.preac2x(a, b, tau, hh) for a, b in zip(R, R0)])
    dr = np.abs(pr - orr)[cond]
    print(f"h {hh}: max |dp_reac| {dr.max():.2e} over {cond.sum()} of 200; p_reac in [{pr.min():.3f}, {pr.max():.3f}]")
    assert cond.sum() > 50 and dr.max() <= 1e-6
    assert (pr >= 0).all() and (pr <= 1).all()
    h.close()
