"""Parity of the HIP path (through the C-ABI) with the FP64 oracle, step by step.

Tolerances (written out here, derived in the design doc):
  * positions: binary32 states with binary64 displacements are bit-identical to
    the oracle's (both round the same binary64 update once); binary64 states
    agree to 1e-12 of the box.  The plain binary32 mode draws its displacements
    through binary32 arithmetic: a coordinate may then round to the binary32
    neighbour of the oracle's, so its moves are held to one binary32 unit of
    the box edge and compared in lock step.
  * pair lists: identical sets; draws bit-identical.
  * p_enc: 1e-12 (FP64), 1e-6 (FP32 with binary64 near-contact arguments);
    the plain FP32 mode reports its error and is held to 1e-4.
  * decisions: identical except draws within 1e-6 of p (counted).
  * propagated radius and p_reac (binary64 on both sides): 1e-9 from identical
    inputs.  The angle of a propagated pair to its old separation (cos Theta,
    drawn from the full propagator on both sides): 1e-8, since both solve
    F(cos Theta) = u to about 1e-12 on coefficients summed in different orders.  In the plain binary32 mode the inputs may differ by one binary32
    unit of a coordinate, i.e. 2^-22 um / sigma = 4.8e-5 in units of sigma at a
    2.5 um box and sigma = 5 nm; R'' and p_reac are then held to 1e-4.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1107_0270_amd import inputs as I
from paper_1107_0270_amd import sim as S

from .parity import make_pair, run

pytestmark = pytest.mark.gpu


def _state(n_a, n_b, box, dim, sigma, seed, f32):
    sp, pos, _ = I.uniform_state(n_a, n_b, box=box, dim=dim, sigma=sigma, seed=seed, f32=f32)
    return sp, pos


def _check(rep, *, p_tol, allow_near=2, rpp_tol=1e-9, cos_tol=1e-8):
    print(rep)
    assert rep.pair_set_mismatch == 0
    assert rep.draw_mismatch == 0
    assert rep.unexplained == 0, rep.notes
    assert rep.max_dp <= p_tol
    assert rep.max_dRpp <= rpp_tol and rep.max_dpreac <= rpp_tol
    assert rep.max_dcos <= cos_tol
    assert rep.near_decisions <= allow_near


def test_abs3d_fp64_trajectory():
    # the 3D absorbing workload in full: 1,000 A + 1,000 B, L = 1 um, 100 steps, FP64
    cfg = I.workload("cfg_abs3d")
    sp, pos = _state(cfg["n_a"], cfg["n_b"], cfg["box"], 3, cfg["sigma"], 0, False)
    gpu, orc = make_pair(dim=3, bc=cfg["bc"], box=cfg["box"], dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"],
                         kappa=0.0, k_off=0.0, precision=S.PREC_FP64, species=sp, pos=pos)
    rep = run(gpu, orc, cfg["steps"], p_tol=1e-12, pos_tol=1e-12, box=cfg["box"])
    _check(rep, p_tol=1e-12)
    assert rep.reactions > 5 and rep.resyncs == 0
    assert gpu.derived()["rcut"] == pytest.approx(orc.derived()["rcut"], rel=1e-12)


KERNELS = [S.PAIRS_BRICKS, S.PAIRS_DIRECT]


F32_ULP_2_5 = 2.0 ** -22  # one binary32 unit in [2, 4): the coordinates of a 2.5 um box


@pytest.mark.parametrize("pair_search", KERNELS)
@pytest.mark.parametrize("prec,p_tol", [(S.PREC_FP32_FP64NC, 1e-6), (S.PREC_FP32, 1e-4)])
def test_rad3d_reversible_binary32(prec, p_tol, pair_search):
    # radiation workload at its density (500 A + 500 B per um^3) in a 2.5 um box;
    # k_off raised so dissociation and geminate recombination occur within the run
    n = 7812
    sp, pos = _state(n, n, 2.5, 3, 0.005, 1, True)
    gpu, orc = make_pair(dim=3, bc=O.BC_RAD, box=2.5, dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, kappa=0.1,
                         k_off=2000.0, precision=prec, species=sp, pos=pos, seed=3, pair_search=pair_search)
    plain = prec == S.PREC_FP32
    rep = run(gpu, orc, 30, p_tol=p_tol, pos_tol=F32_ULP_2_5 if plain else 0.0, box=2.5, lockstep=plain)
    _check(rep, p_tol=p_tol, rpp_tol=1e-4 if plain else 1e-9, cos_tol=1e-3 if plain else 1e-8)
    assert rep.reactions > 20 and rep.decays > 0
    if plain:
        assert rep.max_dmove <= F32_ULP_2_5
        print(f"plain binary32 moves: max |dx| {rep.max_dmove:.3e} um, {rep.pos_resyncs} lock-step reloads in 30 steps")
    else:
        assert rep.max_dmove == 0.0 and rep.pos_resyncs == 0


@pytest.mark.parametrize("dim", [3, 2])
def test_binary32_displacements_stage_parity(dim):
    # FP32D_FP64NC: binary32 Box-Muller displacements, binary64 near-contact pair arithmetic.
    # Its moves differ from the oracle's binary64 ones by binary32 roundings of the
    # displacement, held to 1e-5 of the box.  Stage parity: after each GPU step the oracle takes
    # the GPU's post-move positions and displacements and runs every later stage itself, held
    # to the near-contact mode's bar: pair sets identical, p_enc within 1e-6 (3D; 1e-9 with the
    # binary64 2D expansion), decisions identical but for draws within 1e-6 of p, R'' and p_reac
    # to 1e-9, angles to 1e-8, states after the step bit for bit.
    prec = S.PREC_FP32D_FP64NC
    if dim == 3:
        n, box, steps = 7812, 2.5, 30
        sp, pos = _state(n, n, box, 3, 0.005, 1, True)
        gpu, orc = make_pair(dim=3, bc=O.BC_RAD, box=box, dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, kappa=0.1,
                             k_off=2000.0, precision=prec, species=sp, pos=pos, seed=3)
        p_tol = 1e-6
    else:
        n, box, steps = 3000, 1.5, 8
        sp, pos = _state(n, n, box, 2, 0.005, 7, True)
        gpu, orc = make_pair(dim=2, bc=O.BC_RAD, box=box, dt=5e-6, D=(0.1, 0.1, 0.05), sigma=0.005, kappa=0.05,
                             k_off=2000.0, precision=prec, species=sp, pos=pos, seed=8)
        p_tol = 1e-9
    rep = run(gpu, orc, steps, p_tol=p_tol, pos_tol=0.0, box=box, lockstep=True, stage=True)
    _check(rep, p_tol=p_tol)
    print(f"binary32 displacements: max |dx| against the binary64 move {rep.max_dmove:.3e} um, "
          f"{rep.pos_resyncs} lock-step reloads in {steps} steps")
    assert 0.0 < rep.max_dmove <= 1e-5 * box
    assert rep.matches > 0 and rep.angles > 0


@pytest.mark.parametrize("pair_search", KERNELS)
@pytest.mark.parametrize("cell", [0.0, 0.075])
def test_rad3d_dense(cell, pair_search):
    # a dense, fast system: A's with up to ~16 candidates, chains of several
    # picks per B.  cell = 0.075 um puts ~160 B in every bucket, so the halo of
    # even a one-cell brick overflows LDS and the search reads global memory.
    # (20,000 A + 20,000 B in a 0.375 um box: about 3e5 pairs and 5e4 candidates per step)
    n = 20000
    sp, pos = _state(n, n, 0.375, 3, 0.004, 2, True)
    gpu, orc = make_pair(dim=3, bc=O.BC_RAD, box=0.375, dt=2e-5, D=(5.0, 5.0, 2.5), sigma=0.004, kappa=1.0,
                         k_off=500.0, precision=S.PREC_FP32_FP64NC, species=sp, pos=pos, seed=4, eps_cut=0.05,
                         cell=cell, pair_search=pair_search)
    rep = run(gpu, orc, 5, p_tol=1e-6, pos_tol=0.0, box=0.375)
    _check(rep, p_tol=1e-6, allow_near=3)
    tot = gpu.stats(total=True)
    if cell > 0 and pair_search == S.PAIRS_BRICKS:
        assert tot["lds_fallback"] > 0


def test_reflecting_and_small_box_single_cell():
    # reflecting surface (no reactions, every encounter re-propagated) with one
    # cell for the whole box (the neighbour search then visits that cell once)
    n = 300
    sp, pos = _state(n, n, 0.05, 3, 0.004, 5, False)
    gpu, orc = make_pair(dim=3, bc=O.BC_REF, box=0.05, dt=2e-6, D=(1.0, 1.0, 0.5), sigma=0.004, kappa=0.0,
                         k_off=0.0, precision=S.PREC_FP64, species=sp, pos=pos, seed=6, cell=0.05)
    assert gpu.grid()[3] == 1
    rep = run(gpu, orc, 10, p_tol=1e-12, pos_tol=1e-12, box=0.05)
    _check(rep, p_tol=1e-12)
    assert rep.matches > 0 and rep.reactions == 0


@pytest.mark.parametrize("pair_search", KERNELS)
@pytest.mark.parametrize("prec,p_tol", [(S.PREC_FP64, 1e-12), (S.PREC_FP32_FP64NC, 1e-9)])
def test_mem2d_small_tau(prec, p_tol, pair_search):
    # 2D membrane workload at tau = 0.04 (dt = 5 us), its density (1,250 A and B per um^2)
    n = 7812
    sp, pos = _state(n, n, 2.5, 2, 0.005, 7, prec != S.PREC_FP64)
    gpu, orc = make_pair(dim=2, bc=O.BC_RAD, box=2.5, dt=5e-6, D=(0.1, 0.1, 0.05), sigma=0.005, kappa=0.05,
                         k_off=2000.0, precision=prec, species=sp, pos=pos, seed=8, pair_search=pair_search)
    rep = run(gpu, orc, 20, p_tol=p_tol, pos_tol=0.0 if prec != S.PREC_FP64 else 1e-12, box=2.5)
    _check(rep, p_tol=p_tol)
    assert rep.reactions > 0


def test_mem2d_runtime_order():
    # the 2D step at an expansion order with no compiled form (10): the run-time-order kernels
    n = 3000
    sp, pos = _state(n, n, 1.5, 2, 0.005, 12, False)
    gpu, orc = make_pair(dim=2, bc=O.BC_RAD, box=1.5, dt=5e-6, D=(0.1, 0.1, 0.05), sigma=0.005, kappa=0.05,
                         k_off=2000.0, precision=S.PREC_FP64, species=sp, pos=pos, seed=13, n_terms=10)
    rep = run(gpu, orc, 8, p_tol=1e-12, pos_tol=1e-12, box=1.5)
    _check(rep, p_tol=1e-12)


@pytest.mark.parametrize("pair_search", [S.PAIRS_AUTO, S.PAIRS_BRICKS])
def test_rad3d_full_size_one_step(pair_search):
    # the benchmark workload at full size (1e6 particles, L = 10 um), in the
    # launch configuration the benchmark times (automatic kernel choice) and
    # with the other pair-search kernel
    cfg = I.workload("cfg_rad3d")
    sp, pos = _state(cfg["n_a"], cfg["n_b"], cfg["box"], 3, cfg["sigma"], 0, True)
    gpu, orc = make_pair(dim=3, bc=cfg["bc"], box=cfg["box"], dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"],
                         kappa=cfg["kappa_a"], k_off=cfg["k_off"], precision=cfg["precision"], species=sp, pos=pos,
                         pair_search=pair_search)
    # binary32 displacements: stage parity (the oracle continues from the GPU's own move)
    rep = run(gpu, orc, 2, p_tol=1e-6, pos_tol=0.0, box=cfg["box"], stage=cfg["precision"] == S.PREC_FP32D_FP64NC)
    _check(rep, p_tol=1e-6)
    assert rep.pairs > 10000


@pytest.mark.parametrize("name,p_tol", [("cfg_rad3d_dense", 1e-6)])
def test_full_size_many_events(name, p_tol):
    # full-size workloads with thousands of encounters per step: the event kernel
    # runs one event per lane there (4096 or more events)
    cfg = I.workload(name)
    sp, pos = _state(cfg["n_a"], cfg["n_b"], cfg["box"], cfg["dim"], cfg["sigma"], 0, True)
    gpu, orc = make_pair(dim=cfg["dim"], bc=cfg["bc"], box=cfg["box"], dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"],
                         kappa=cfg["kappa_a"], k_off=cfg["k_off"], precision=cfg["precision"], species=sp, pos=pos)
    rep = run(gpu, orc, 1, p_tol=p_tol, pos_tol=0.0, box=cfg["box"], stage=cfg["precision"] == S.PREC_FP32D_FP64NC)
    _check(rep, p_tol=p_tol, allow_near=4)
    st = gpu.stats()
    print("events", st["matches"] + st["decay"])
    assert st["matches"] + st["decay"] >= 4096


def test_cell_lists_are_consistent():
    # every live slot is binned once, in the bucket of its post-move position
    n = 5000
    sp, pos = _state(n, n, 1.0, 3, 0.005, 11, True)
    gpu, _ = make_pair(dim=3, bc=O.BC_RAD, box=1.0, dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, kappa=0.1,
                       k_off=10.0, precision=S.PREC_FP32_FP64NC, species=sp, pos=pos)
    sp0 = gpu.species()
    gpu.step()
    keys, moved = gpu.dbg_cells(), gpu.dbg_moved()
    nx, ny, nz, ncell, _ = gpu.grid()
    live = sp0 <= S.SP_C
    c = [np.clip(np.floor(moved[live, k] * (m / 1.0)).astype(np.int64), 0, m - 1) for k, m in enumerate((nx, ny, nz))]
    expect = sp0[live].astype(np.int64) * ncell + (c[2] * ny + c[1]) * nx + c[0]
    assert np.array_equal(keys[live].astype(np.int64), expect)
    assert np.all(keys[~live] == 0xFFFFFFFF)


def test_degenerate_inputs():
    # no B at all; a single A; all slots free except one C with its reserved slot
    box = 1.0
    sp = np.zeros(10, np.int32)
    pos = np.random.default_rng(0).random((10, 3))
    g = S.Sim(dim=3, box=box, dt=1e-6, D=(1.0, 1.0, 0.5), sigma=0.005, bc=S.BC_ABSORBING, species=sp, pos=pos,
              precision=S.PREC_FP64)
    g.step(3)
    assert g.counts()["A"] == 10 and g.stats()["pairs"] == 0
    g1 = S.Sim(dim=2, box=box, dt=5e-7, D=(1.0, 1.0, 0.5), sigma=0.005, bc=S.BC_RADIATION, kappa=0.1,
               species=np.array([0], np.int32), pos=np.array([[0.5, 0.5]]))
    g1.step(2)
    assert g1.counts()["A"] == 1
    sp = np.array([2, 4, 3], np.int32)
    pos = np.array([[0.5, 0.5, 0.5], [0, 0, 0], [0, 0, 0]], float)
    gc, oc = make_pair(dim=3, bc=O.BC_RAD, box=box, dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, kappa=0.1,
                       k_off=3e4, precision=S.PREC_FP64, species=sp, pos=pos, partner=np.array([1, 0xFFFFFFFF, 0xFFFFFFFF], np.uint32))
    rep = run(gc, oc, 40, p_tol=1e-12, pos_tol=1e-12, box=box)
    _check(rep, p_tol=1e-12)
    assert rep.decays > 0


def test_rad3d_unequal_diffusion_constants():
    # D_A != D_B: the placement weights D_A / D_eff, D_B / D_eff of eq. Rcoo, for the
    # propagated pairs (their angle drawn), the products of a reaction and of a decay
    n = 2500
    sp, pos = _state(n, n, 1.0, 3, 0.005, 23, False)
    gpu, orc = make_pair(dim=3, bc=O.BC_RAD, box=1.0, dt=1e-5, D=(0.4, 1.6, 0.32), sigma=0.005, kappa=0.1,
                         k_off=3000.0, precision=S.PREC_FP64, species=sp, pos=pos, seed=29)
    rep = run(gpu, orc, 12, p_tol=1e-12, pos_tol=1e-12, box=1.0)
    _check(rep, p_tol=1e-12)
    assert rep.angles > 50 and rep.decays > 0 and rep.reactions > 0


def test_keep_direction_flag_matches_the_oracle_reading():
    # SIM_F_KEEP_DIRECTION: the propagated pair keeps its free end point's direction, on both
    # sides (no angle is drawn, cos Theta stays NaN in the logs)
    n = 3000
    sp, pos = _state(n, n, 1.25, 3, 0.005, 31, True)
    gpu, orc = make_pair(dim=3, bc=O.BC_RAD, box=1.25, dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, kappa=0.1,
                         k_off=2000.0, precision=S.PREC_FP32_FP64NC, species=sp, pos=pos, seed=5, keep_direction=True)
    rep = run(gpu, orc, 8, p_tol=1e-6, pos_tol=0.0, box=1.25)
    _check(rep, p_tol=1e-6)
    assert rep.matches > 20 and rep.angles == 0


def _u(w):
    return (np.asarray(w, np.float64) + 0.5) * 2.0 ** -32


def test_membrane_as_written_full_size_sampled():
    # The membrane workload as written at full size (10^6 particles, tau = 0.8, exact 2D
    # functions) in the benchmark's launch configuration (pair cut-off 1e-6): one GPU step with
    # its stage logs, checked on samples the oracle computes one by one (the whole step would
    # take the oracle minutes): p_enc and the candidate draws of 400 pairs, R'', p_reac and the
    # reaction draws of 300 matches, the angle of 150 propagated pairs, and the placements.
    cfg = I.workload("cfg_mem2d")
    sp, pos = _state(cfg["n_a"], cfg["n_b"], cfg["box"], 2, cfg["sigma"], 0, True)
    gpu = S.Sim(dim=2, box=cfg["box"], dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"], bc=cfg["bc"],
                kappa=cfg["kappa_a"], k_off=cfg["k_off"], precision=cfg["precision"], species=sp, pos=pos,
                green2d=S.G2_EXACT, eps_cut=1e-6, debug=True, debug_cap=1 << 22)
    d = gpu.derived()
    tau, hh, a = d["tau"], d["hh"], d["a"]
    key, step = (0, 0), 0
    gpu.step()
    st = gpu.stats()
    print("pairs", st["pairs"], "matches", st["matches"], "decays", st["decay"])
    assert st["matches"] + st["decay"] >= 4096  # one event per lane
    gp, gm = gpu.dbg_pairs(), gpu.dbg_matches()
    assert len(gp) == st["pairs"] and len(gm) == st["matches"]
    rng = np.random.default_rng(4)
    sw, swp = O.x2_switch(tau), O.x2_prop_switch(tau)
    # pairs: p_enc, draws, candidate decisions
    for r in gp[rng.choice(len(gp), 400, replace=False)]:
        i, j = int(r["i"]), int(r["j"])
        R, R0 = float(r["R"]), float(r["R0"])
        want = 1.0 if R <= 1.0 else (O.penc2x(R, R0, tau) if R0 <= sw else O.penc2(R, R0, tau, 12))
        assert abs(r["p"] - want) <= 1e-6, (i, j, R, R0, r["p"], want)
        assert int(r["draw"]) == int(O.philox((i, j, step, 2), key)[0])
        assert bool(r["cand"]) == (R <= 1.0 or _u(r["draw"]) < r["p"])
    # matches: R'', p_reac, reaction draws, angles
    R0_of = {(int(r["i"]), int(r["j"])): float(r["R0"]) for r in gp}
    n_ang = 0
    for r in gm[rng.choice(len(gm), 300, replace=False)]:
        i, j = int(r["i"]), int(r["j"])
        R0, Rpp = max(R0_of[(i, j)], 1.0), float(r["Rpp"])
        if R0 <= swp:
            u = _u(O.philox((i, j, step, 5), key)[0])
            assert abs(Rpp - O.sample_prop2x(R0, tau, u)) <= 1e-5
        else:
            Ro, ao, _ = O.sample_prop(2, R0, tau, 12, (i, j, step, 5), key)
            assert abs(Rpp - Ro) <= 1e-9 and r["attempts"] == ao
        want = O.preac2x(Rpp, R0, tau, hh) if R0 <= sw else O.preac2(Rpp, R0, tau, hh, 12)
        assert abs(r["preac"] - want) <= 1e-6
        assert int(r["draw"]) == int(O.philox((i, j, step, 6), key)[0])
        assert bool(r["reacted"]) == (_u(r["draw"]) < r["preac"])
        if r["reacted"]:
            assert np.isnan(r["cos_theta"])
            continue
        if n_ang < 150:  # the angle solves the oracle's distribution function at its uniform
            n_ang += 1
            u = _u(O.philox((i, j, step, 13), key)[0])
            w = O.angle2_coef(0, max(Rpp, 1.0), R0, tau)
            th = math.acos(min(1.0, max(-1.0, float(r["cos_theta"]))))
            tol = 1e-9 + 1e-14 * math.exp((max(Rpp, 1.0) + R0 - 2.0) ** 2 / (4.0 * tau))
            assert abs(O.angle2_cdf(w, th) - u) < tol, (i, j, Rpp, R0, u, th)
    assert n_ang >= 100
    # placements: every propagated pair sits a R'' apart
    spn, x, _ = gpu.state()
    box = cfg["box"]
    prop = gm[gm["reacted"] == 0]
    dv = x[prop["j"].astype(np.int64)] - x[prop["i"].astype(np.int64)]
    dv -= box * np.round(dv / box)
    sep = np.linalg.norm(dv, axis=1) / a
    assert np.abs(sep - prop["Rpp"]).max() < 2e-3  # binary32 coordinates of a 20 um box: 1e-6 um / 5 nm
    gpu.close()
