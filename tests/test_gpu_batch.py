"""Batches of independent replicas: every replica of a batch must follow exactly the trajectory
it follows alone (same draws, same arithmetic), whatever the other replicas are, and a replica is
held to the oracle directly, stage by stage (test_a_batch_member_follows_the_oracle)."""
import numpy as np
import pytest

from paper_1107_0270_amd import inputs as I
from paper_1107_0270_amd import sim as S

pytestmark = pytest.mark.gpu

SHARED = dict(dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, bc=S.BC_RADIATION, k_off=2000.0, seed=21)


def _replicas(counts, prec, seed=5):
    rng = np.random.default_rng(seed)
    reps = []
    for r, n in enumerate(counts):
        box = float(np.float32((n / 1000.0) ** (1.0 / 3.0)))  # the density of 500 A + 500 B per um^3
        sp, pos, _ = I.uniform_state(n // 2, n - n // 2, box=box, dim=3, sigma=0.005, seed=100 + r,
                                     f32=prec != S.PREC_FP64)
        reps.append(dict(species=sp, pos=pos, box=box, kappa=float(rng.uniform(0.01, 1.0)), replica=7 + 3 * r))
    return reps


def _alone(rd, prec, steps, pair_search=S.PAIRS_AUTO):
    sim = S.Sim(dim=3, box=rd["box"], species=rd["species"], pos=rd["pos"], kappa=rd["kappa"], replica=rd["replica"],
                precision=prec, pair_search=pair_search, **SHARED)
    sim.step(steps)
    sp, pos, pt = sim.state()
    st = sim.stats(total=True)
    sim.close()
    return sp, pos, pt, st


@pytest.mark.parametrize("prec", [S.PREC_FP32_FP64NC, S.PREC_FP64])
def test_each_replica_of_a_batch_runs_as_it_runs_alone(prec):
    counts = [600, 2200, 1000, 3400, 1500]
    reps = _replicas(counts, prec)
    steps = 15
    b = S.Sim.batch(reps, precision=prec, **SHARED)
    b.step(steps)
    sp, pos, pt = b.state()
    tot = b.stats(total=True)
    sums = {k: 0 for k in ("pairs", "matches", "react", "decay", "geminate")}
    for r, rd in enumerate(reps):
        lo, hi = b.slot_base[r], b.slot_base[r] + counts[r]
        sp1, pos1, pt1, st1 = _alone(rd, prec, steps)
        assert np.array_equal(sp[lo:hi], sp1), f"replica {r}: species differ"
        live = sp1 <= S.SP_C
        d = np.abs(pos[lo:hi][live] - pos1[live])
        assert d.max() <= (0.0 if prec != S.PREC_FP64 else 1e-12), f"replica {r}: positions differ by {d.max()}"
        c = sp1 == S.SP_C
        assert np.array_equal(pt[lo:hi][c].astype(np.int64) - lo, pt1[c].astype(np.int64)), f"replica {r}: partners"
        for k in sums:
            sums[k] += st1[k]
        print(f"replica {r}: n {counts[r]} kappa {rd['kappa']:.3f} reactions {st1['react']} decays {st1['decay']}")
    for k in sums:
        assert tot[k] == sums[k], (k, tot[k], sums[k])
    assert sums["react"] > 0 and sums["decay"] > 0
    b.close()


def test_batch_of_one_is_the_single_system():
    reps = _replicas([4000], S.PREC_FP32_FP64NC, seed=9)
    b = S.Sim.batch(reps, precision=S.PREC_FP32_FP64NC, **SHARED)
    b.step(10)
    sp, pos, pt = b.state()
    sp1, pos1, pt1, _ = _alone(reps[0], S.PREC_FP32_FP64NC, 10, pair_search=S.PAIRS_DIRECT)
    assert np.array_equal(sp, sp1)
    live = sp1 <= S.SP_C
    assert np.array_equal(pos[live], pos1[live])
    b.close()


def test_2d_batch_replicas_run_as_alone():
    shared2 = dict(dim=2, dt=5e-6, D=(0.1, 0.1, 0.05), sigma=0.005, bc=S.BC_RADIATION, k_off=2000.0, seed=3,
                   precision=S.PREC_FP32_FP64NC)
    rng = np.random.default_rng(2)
    reps = []
    for r, n in enumerate([1500, 4000, 2500]):
        box = float(np.float32((n / 1250.0) ** 0.5))
        sp, pos, _ = I.uniform_state(n // 2, n - n // 2, box=box, dim=2, sigma=0.005, seed=50 + r, f32=True)
        reps.append(dict(species=sp, pos=pos, box=box, kappa=float(rng.uniform(0.01, 0.1)), replica=r))
    b = S.Sim.batch(reps, **shared2)
    b.step(12)
    sp, pos, pt = b.state()
    for r, rd in enumerate(reps):
        kw = dict(shared2)
        kw.pop("dim")
        a = S.Sim(dim=2, box=rd["box"], species=rd["species"], pos=rd["pos"], kappa=rd["kappa"], replica=rd["replica"], **kw)
        a.step(12)
        sp1, pos1, pt1 = a.state()
        a.close()
        lo, hi = b.slot_base[r], b.slot_base[r] + len(rd["species"])
        assert np.array_equal(sp[lo:hi], sp1)
        live = sp1 <= S.SP_C
        assert np.array_equal(pos[lo:hi][live], pos1[live])
    b.close()


def test_replicas_joining_at_their_own_steps():
    # a replica continued inside a batch from a state read at its step s follows the
    # uninterrupted trajectory: the draws are keyed on its own step
    prec = S.PREC_FP32_FP64NC
    reps = _replicas([1200, 2600, 1800], prec, seed=11)
    # uninterrupted runs: 10 steps each
    ref = [_alone(rd, prec, 10) for rd in reps]
    # replica r first runs alone for s_r steps, then all continue together
    pre = [3, 0, 7]
    cont = []
    for rd, s in zip(reps, pre):
        a = S.Sim(dim=3, box=rd["box"], species=rd["species"], pos=rd["pos"], kappa=rd["kappa"], replica=rd["replica"],
                  precision=prec, **SHARED)
        a.step(s)
        sp, pos, pt = a.state()
        a.close()
        cont.append(dict(rd, species=sp, pos=pos, partner=np.where(sp == S.SP_C, pt, 0xFFFFFFFF), step=s))
    # the batch steps until replica 1 (no head start) has 10 steps; others get extra runs below
    b = S.Sim.batch(cont, precision=prec, **SHARED)
    b.step(3)
    sp, pos, pt = b.state()
    # replica 2 has now done 7 + 3 = 10 steps
    lo, hi = b.slot_base[2], b.slot_base[2] + 1800
    assert np.array_equal(sp[lo:hi], ref[2][0])
    live = ref[2][0] <= S.SP_C
    assert np.array_equal(pos[lo:hi][live], ref[2][1][live])
    b.step(4)
    sp, pos, pt = b.state()
    lo, hi = b.slot_base[0], b.slot_base[0] + 1200  # 3 + 7 = 10 steps
    assert np.array_equal(sp[lo:hi], ref[0][0])
    live = ref[0][0] <= S.SP_C
    assert np.array_equal(pos[lo:hi][live], ref[0][1][live])
    b.step(3)
    sp, pos, pt = b.state()
    lo, hi = b.slot_base[1], b.slot_base[1] + 2600  # 0 + 10 steps
    assert np.array_equal(sp[lo:hi], ref[1][0])
    live = ref[1][0] <= S.SP_C
    assert np.array_equal(pos[lo:hi][live], ref[1][1][live])
    c = ref[1][0] == S.SP_C
    assert np.array_equal(pt[lo:hi][c].astype(np.int64) - lo, ref[1][2][c].astype(np.int64))
    b.close()


@pytest.mark.parametrize("dim", [3, 2])
def test_a_batch_member_follows_the_oracle(dim):
    # One replica of a batch (its own kappa, box and Philox key) in lock step with the oracle's
    # step of that replica alone (OracleSim(replica=r)): after every step the batch's stage logs
    # restricted to the replica's slots (post-move positions, pairs with p_enc and draws, picks,
    # matches with R'', p_reac and the angle, dissociations) and its state are compared with the
    # oracle's, to the tolerances of the single-system parity tests.
    import oracle as O
    from . import parity as PT

    prec = S.PREC_FP32_FP64NC
    if dim == 3:
        shared = dict(SHARED)
        counts = [1200, 2600, 1800]
        reps = _replicas(counts, prec, seed=11)
    else:
        shared = dict(dt=5e-6, D=(0.1, 0.1, 0.05), sigma=0.005, bc=S.BC_RADIATION, k_off=2000.0, seed=3)
        counts = [900, 1600, 1100]
        reps = []
        for r, n in enumerate(counts):
            box = float(np.float32((n / 1250.0) ** 0.5))
            sp, pos, _ = I.uniform_state(n // 2, n - n // 2, box=box, dim=2, sigma=0.005, seed=70 + r, f32=True)
            reps.append(dict(species=sp, pos=pos, box=box, kappa=0.02 + 0.03 * r, replica=4 + r))
    b = S.Sim.batch(reps, dim=dim, precision=prec, debug=True, debug_cap=1 << 20, eps_cut=1e-3, **shared)
    r = 1
    rd = reps[r]
    view = PT.MemberView(b, b.slot_base[r], counts[r])
    orc = O.OracleSim(dim=dim, bc=shared["bc"], box=[rd["box"]] * dim, dt=shared["dt"], D=shared["D"],
                      sigma=shared["sigma"], kappa_a=rd["kappa"], k_off=shared["k_off"], eps_cut=1e-3,
                      seed=shared["seed"], replica=rd["replica"], store_f32=True, species=rd["species"], pos=rd["pos"])
    rep = PT.run(view, orc, 24 if dim == 3 else 6, p_tol=1e-6 if dim == 3 else 1e-9, pos_tol=0.0, box=rd["box"],
                 lockstep=False)
    print(rep)
    assert rep.unexplained == 0, rep.notes
    assert rep.resyncs == 0
    assert rep.pair_set_mismatch == 0 and rep.draw_mismatch == 0
    assert rep.near_decisions <= 2
    assert rep.max_dp <= (1e-6 if dim == 3 else 1e-9)
    assert rep.max_dRpp <= 1e-9 and rep.max_dpreac <= 1e-9
    assert rep.max_dcos <= 1e-8
    assert rep.matches > 0 and rep.angles > 0
    b.close()


def test_2d_exact_batch_replicas_run_as_alone():
    # tau = 0.8: the batch builds exact 2D tables per distinct kappa (replicas 0 and 2 share a
    # set) and every replica follows its single-system trajectory (exact tables too) bit for bit
    shared2 = dict(dim=2, dt=1e-4, D=(0.1, 0.1, 0.05), sigma=0.005, bc=S.BC_RADIATION, k_off=2000.0, seed=3,
                   precision=S.PREC_FP32_FP64NC, green2d=S.G2_EXACT)
    reps = []
    for r, (n, kappa) in enumerate([(1000, 0.05), (1500, 0.1), (1200, 0.05)]):
        box = float(np.float32((n / 1250.0) ** 0.5))
        sp, pos, _ = I.uniform_state(n // 2, n - n // 2, box=box, dim=2, sigma=0.005, seed=80 + r, f32=True)
        reps.append(dict(species=sp, pos=pos, box=box, kappa=kappa, replica=r))
    b = S.Sim.batch(reps, **shared2)
    b.step(8)
    sp, pos, pt = b.state()
    for r, rd in enumerate(reps):
        kw = dict(shared2)
        kw.pop("dim")
        a = S.Sim(dim=2, box=rd["box"], species=rd["species"], pos=rd["pos"], kappa=rd["kappa"], replica=rd["replica"], **kw)
        a.step(8)
        sp1, pos1, pt1 = a.state()
        st = a.stats(total=True)
        a.close()
        lo, hi = b.slot_base[r], b.slot_base[r] + len(rd["species"])
        assert np.array_equal(sp[lo:hi], sp1), f"replica {r}"
        live = sp1 <= S.SP_C
        assert np.array_equal(pos[lo:hi][live], pos1[live]), f"replica {r}"
        print(f"replica {r}: matches {st['matches']} reactions {st['react']}")
    b.close()
