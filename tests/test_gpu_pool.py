"""Pools (continuous batching): systems join a running pool and leave it between steps, and
every member follows exactly the trajectory it follows alone, whenever it joined, whoever
shared the pool and wherever its slots landed (including slots freed by a member that left).
A member that joins a running pool is held to the oracle directly, stage by stage
(test_a_pool_member_follows_the_oracle)."""
import numpy as np
import pytest

from paper_1107_0270_amd import inputs as I
from paper_1107_0270_amd import sim as S

pytestmark = pytest.mark.gpu

SHARED3 = dict(dim=3, dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, bc=S.BC_RADIATION, k_off=2000.0, seed=21)
SHARED2 = dict(dim=2, dt=5e-6, D=(0.1, 0.1, 0.05), sigma=0.005, bc=S.BC_RADIATION, k_off=2000.0, seed=3)


def _system(n, dim, seed, density, prec=S.PREC_FP32_FP64NC, kappa=0.3, replica=0):
    box = float(np.float32((n / density) ** (1.0 / dim)))
    sp, pos, _ = I.uniform_state(n // 2, n - n // 2, box=box, dim=dim, sigma=0.005, seed=seed, f32=prec != S.PREC_FP64)
    return dict(species=sp, pos=pos, box=box, kappa=kappa, replica=replica)


def _alone(sd, shared, prec, steps):
    sim = S.Sim(box=sd["box"], species=sd["species"], pos=sd["pos"], kappa=sd["kappa"], replica=sd["replica"],
                precision=prec, **shared)
    sim.step(steps)
    out = sim.state()
    sim.close()
    return out


def _same(got, want, prec, what):
    sp, pos, pt = got
    sp1, pos1, pt1 = want
    assert np.array_equal(sp, sp1), f"{what}: species differ"
    live = sp1 <= S.SP_C
    d = np.abs(pos[live] - pos1[live])
    assert d.size == 0 or d.max() <= (0.0 if prec != S.PREC_FP64 else 1e-12), f"{what}: positions differ by {d.max()}"
    c = sp1 == S.SP_C
    assert np.array_equal(pt[c], pt1[c]), f"{what}: partners differ"
    return int(c.sum())


def _pool(shared, prec, slot_cap, **kw):
    sh = dict(shared)
    dim = sh.pop("dim")
    return S.Pool(dim=dim, box=1.0, slot_cap=slot_cap, precision=prec, **sh, **kw)


@pytest.mark.parametrize("prec", [S.PREC_FP32_FP64NC, S.PREC_FP64])
def test_members_joining_and_leaving_run_as_alone(prec):
    a = _system(5000, 3, 11, 1000.0, prec, kappa=0.2, replica=1)
    b = _system(4000, 3, 12, 1000.0, prec, kappa=0.7, replica=2)
    c = _system(5000, 3, 13, 1000.0, prec, kappa=0.05, replica=3)
    # room for a and b only: c reuses a's slots, and its records need the dead ones dropped
    pool = _pool(SHARED3, prec, slot_cap=9500)
    ma = pool.admit(**a)
    pool.step(7)
    mb = pool.admit(**b)
    pool.step(5)
    n_c = _same(pool.member_state(ma), _alone(a, SHARED3, prec, 12), prec, "a after 12 steps")
    pool.retire(ma)
    mc = pool.admit(**c)  # first fit: a's slots
    assert pool.try_admit(**_system(600, 3, 99, 1000.0, prec)) is None  # 500 free slots left
    assert pool.try_admit(**_system(400, 3, 98, 1000.0, prec)) is not None
    pool.step(9)
    n_c += _same(pool.member_state(mb), _alone(b, SHARED3, prec, 14), prec, "b after 14 steps")
    n_c += _same(pool.member_state(mc), _alone(c, SHARED3, prec, 9), prec, "c after 9 steps")
    pool.retire(mb)
    pool.step(4)
    n_c += _same(pool.member_state(mc), _alone(c, SHARED3, prec, 13), prec, "c after 13 steps")
    assert n_c > 0  # reactions happened
    pool.close()


def test_2d_pool_members_run_as_alone():
    prec = S.PREC_FP32_FP64NC
    a = _system(3000, 2, 21, 2500.0, prec, kappa=0.05, replica=5)
    b = _system(2000, 2, 22, 2500.0, prec, kappa=0.02, replica=6)
    pool = _pool(SHARED2, prec, slot_cap=6000)
    ma = pool.admit(**a)
    pool.step(4)
    mb = pool.admit(**b)
    pool.step(6)
    _same(pool.member_state(ma), _alone(a, SHARED2, prec, 10), prec, "2D a")
    _same(pool.member_state(mb), _alone(b, SHARED2, prec, 6), prec, "2D b")
    pool.close()


def test_dense_member_after_sparse_ones():
    # a sparse member allows the narrow pair search; a dense one needs the general one, and the
    # pool's step graphs are rebuilt for it
    prec = S.PREC_FP32_FP64NC
    sparse = _system(2000, 3, 31, 300.0, prec, replica=8)
    dense = _system(6000, 3, 32, 40000.0, prec, replica=9)
    pool = _pool(SHARED3, prec, slot_cap=8000)
    ms = pool.admit(**sparse)
    pool.step(3)
    md = pool.admit(**dense)
    pool.step(5)
    _same(pool.member_state(ms), _alone(sparse, SHARED3, prec, 8), prec, "sparse")
    _same(pool.member_state(md), _alone(dense, SHARED3, prec, 5), prec, "dense")
    pool.close()


def test_member_continued_at_its_own_step():
    prec = S.PREC_FP32_FP64NC
    a = _system(4000, 3, 41, 1000.0, prec, kappa=1.0, replica=4)
    sim = S.Sim(box=a["box"], species=a["species"], pos=a["pos"], kappa=a["kappa"], replica=a["replica"],
                precision=prec, **SHARED3)
    sim.step(6)
    sp, pos, pt = sim.state()
    sim.close()
    assert (sp == S.SP_C).any()
    pool = _pool(SHARED3, prec, slot_cap=5000)
    pool.step(2)  # the pool's own counter is ahead of the member's
    m = pool.admit(species=sp, pos=pos, box=a["box"], kappa=a["kappa"], replica=a["replica"], step=6,
                   partner=np.where(sp == S.SP_C, pt, 0xFFFFFFFF).astype(np.uint32))
    pool.step(5)
    _same(pool.member_state(m), _alone(a, SHARED3, prec, 11), prec, "continued member")
    cnt = pool.member_counts(m)
    assert cnt["A"] + cnt["B"] + 2 * cnt["C"] == 4000
    pool.close()


def test_pool_errors_and_capacity():
    prec = S.PREC_FP32_FP64NC
    pool = _pool(SHARED3, prec, slot_cap=3000, rep_cap=2)
    pool.step(2)  # an empty pool steps
    with pytest.raises(S.SimError) as e:
        pool.admit(**_system(3001, 3, 1, 1000.0, prec))
    assert e.value.code == S.SIM_ECAPACITY
    m1 = pool.admit(**_system(1000, 3, 2, 1000.0, prec))
    m2 = pool.admit(**_system(1000, 3, 3, 1000.0, prec))
    assert pool.try_admit(**_system(500, 3, 4, 1000.0, prec)) is None  # both member entries taken
    pool.retire(m1)
    with pytest.raises(S.SimError) as e:
        pool.retire(m1)
    assert e.value.code == S.SIM_EINVAL
    with pytest.raises(S.SimError) as e:
        pool._read_member(m1, S.READ_POS, np.zeros(3000))
    assert e.value.code == S.SIM_EINVAL
    with pytest.raises(S.SimError) as e:
        pool._read_member(m2, S.READ_STATS, np.zeros(64))
    assert e.value.code == S.SIM_EINVAL
    with pytest.raises(S.SimError) as e:
        pool.load_state(0, np.zeros(3000, np.int32), np.zeros((3000, 3)))
    assert e.value.code == S.SIM_ESTATE
    bad = _system(1000, 3, 5, 1000.0, prec)
    bad["pos"] = bad["pos"].copy()
    bad["pos"][0, 0] = np.nan
    with pytest.raises(S.SimError) as e:
        pool.admit(**bad)
    assert e.value.code == S.SIM_EINVAL
    pool.step(3)
    pool.close()
    single = S.Sim(box=1.0, species=np.zeros(10, np.int32), pos=np.full((10, 3), 0.5), precision=prec, **{k: v for k, v in SHARED3.items() if k != "dim"}, dim=3)
    rep = S.SimReplica()
    m = S.C.c_uint32(0)
    assert S.lib().sim_pool_admit(single._h, S.C.byref(rep), S.C.byref(m)) == S.SIM_ESTATE
    assert S.lib().sim_pool_retire(single._h, 0) == S.SIM_ESTATE
    single.close()


def test_a_pool_member_follows_the_oracle():
    # A member that joins a running pool (own kappa, box, Philox key, its own step counter
    # starting at 0 while the pool is at step 5) in lock step with the oracle's step of that
    # system alone (OracleSim(replica=r)): stage logs restricted to the member's slots and its
    # state after every step, to the tolerances of the single-system parity tests.
    import oracle as O
    from . import parity as PT

    prec = S.PREC_FP32_FP64NC
    x = _system(3000, 3, 31, 1000.0, prec, kappa=0.5, replica=2)
    y = _system(2400, 3, 32, 1000.0, prec, kappa=0.1, replica=9)
    pool = _pool(SHARED3, prec, slot_cap=8000, debug=True, debug_cap=1 << 20, eps_cut=1e-3)
    pool.admit(**x)
    pool.step(5)
    my = pool.admit(**y)
    # the member's slots in the pool: the first free range after x's (checked against its own read)
    lo = 3000
    sp_m, pos_m, _ = pool.member_state(my)
    sp_all, pos_all, _ = pool.state()
    assert np.array_equal(sp_all[lo:lo + 2400], sp_m) and np.array_equal(pos_all[lo:lo + 2400], pos_m)
    view = PT.MemberView(pool, lo, 2400)
    sh = dict(SHARED3)
    orc = O.OracleSim(dim=3, bc=sh["bc"], box=[y["box"]] * 3, dt=sh["dt"], D=sh["D"], sigma=sh["sigma"],
                      kappa_a=y["kappa"], k_off=sh["k_off"], eps_cut=1e-3, seed=sh["seed"], replica=y["replica"],
                      store_f32=True, species=y["species"], pos=y["pos"])
    rep = PT.run(view, orc, 20, p_tol=1e-6, pos_tol=0.0, box=y["box"], lockstep=False)
    print(rep)
    assert rep.unexplained == 0, rep.notes
    assert rep.resyncs == 0
    assert rep.pair_set_mismatch == 0 and rep.draw_mismatch == 0
    assert rep.near_decisions <= 2
    assert rep.max_dp <= 1e-6 and rep.max_dRpp <= 1e-9 and rep.max_dpreac <= 1e-9 and rep.max_dcos <= 1e-8
    assert rep.matches > 0 and rep.angles > 0
    pool.close()


def test_2d_exact_pool_member_follows_the_oracle():
    # The membrane workload as written (tau = 0.8) needs the exact 2D tables (the expansion is
    # refused there).  A pool builds them per member kappa (members with equal kappa share a
    # set); a member that joins the running pool is held to the oracle's exact step of its own
    # system.  binary64 state: R'' comes from interpolated tables, so products may land ~1e-9 um
    # from the oracle's, held to 1e-7 um without reloading.
    import oracle as O
    from . import parity as PT

    prec = S.PREC_FP64
    sh = dict(SHARED2, dt=1e-4)
    x = _system(1400, 2, 41, 2500.0, prec, kappa=0.05, replica=3)
    y = _system(1200, 2, 42, 2500.0, prec, kappa=0.2, replica=8)
    pool = _pool(sh, prec, slot_cap=4000, debug=True, debug_cap=1 << 20, eps_cut=1e-3, green2d=S.G2_EXACT)
    pool.admit(**x)
    pool.step(3)
    my = pool.admit(**y)
    lo = 1400
    sp_m, pos_m, _ = pool.member_state(my)
    sp_all, pos_all, _ = pool.state()
    assert np.array_equal(sp_all[lo:lo + 1200], sp_m) and np.array_equal(pos_all[lo:lo + 1200], pos_m)
    view = PT.MemberView(pool, lo, 1200)
    orc = O.OracleSim(dim=2, bc=sh["bc"], box=[y["box"]] * 2, dt=sh["dt"], D=sh["D"], sigma=sh["sigma"],
                      kappa_a=y["kappa"], k_off=sh["k_off"], eps_cut=1e-3, seed=sh["seed"], replica=y["replica"],
                      store_f32=False, exact2d=True, species=y["species"], pos=y["pos"])
    rep = PT.run(view, orc, 6, p_tol=1e-6, pos_tol=1e-7, box=y["box"], lockstep=False)
    print(rep)
    assert rep.unexplained == 0, rep.notes
    assert rep.resyncs == 0
    assert rep.pair_set_mismatch == 0 and rep.draw_mismatch == 0
    assert rep.near_decisions <= 2
    assert rep.max_dp <= 1e-6 and rep.max_dRpp <= 1e-4 and rep.max_dpreac <= 1e-6
    assert rep.matches > 0 and rep.angles > 0
    # the pool's own kernel-level evaluation has no tables of its own: refused, not approximated
    with pytest.raises(S.SimError):
        pool.eval_pairs(np.array([1.1]), np.array([1.2]))
    pool.close()
