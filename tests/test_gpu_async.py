"""sim_step_async enqueues the same steps as sim_step (Sec. 3: a step reads only the device
state the previous one left) without waiting for them; sim_sync waits and reports the
per-step buffer flags.  Checked through the C-ABI: a handle stepped asynchronously, in
several calls, with host work between them, ends in the state of one stepped
synchronously, bit for bit (species, binary32 positions, partners), for a single 3D system,
a 2D one and a pool; reads after asynchronous steps see every one of them; handles that log
or time every step refuse the call."""
import numpy as np
import pytest

from paper_1107_0270_amd import inputs as I
from paper_1107_0270_amd import sim as S

from .test_gpu_pool import SHARED3, _pool, _same, _system

pytestmark = pytest.mark.gpu


def _handle(dim, **kw):
    # the 3D radiation workload at 1.2e5 particles in a 5 um box (binary32 displacements);
    # 2D: the membrane workload at tau = 0.04 on a 6 um square (binary32, expansion of order 12)
    if dim == 3:
        cfg = I.workload("cfg_rad3d", n_a=60_000, n_b=60_000, box=5.0)
    else:
        cfg = I.workload("cfg_mem2d_small_tau", n_a=45_000, n_b=45_000, box=6.0)
    sp, pos, _ = I.uniform_state(cfg["n_a"], cfg["n_b"], box=cfg["box"], dim=dim, sigma=cfg["sigma"], seed=5)
    return S.Sim(dim=dim, box=cfg["box"], dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"], bc=cfg["bc"],
                 kappa=cfg["kappa_a"], k_off=cfg["k_off"], precision=cfg["precision"], species=sp, pos=pos, **kw)


@pytest.mark.parametrize("dim", [3, 2])
def test_async_steps_equal_synchronous_steps(dim):
    a, b = _handle(dim), _handle(dim)
    a.step(24)
    for k in (1, 7, 16):  # 24 steps in three calls, host work between them
        b.step_async(k)
        np.sort(np.random.default_rng(k).random(200_000))
    b.sync()
    got, want = b.state(), a.state()
    n_c = _same(got, want, S.PREC_FP32_FP64NC, f"{dim}D")
    st_a, st_b = a.stats(total=True), b.stats(total=True)
    print(dim, "C", n_c, "pairs", st_a["pairs"], "matches", st_a["matches"])
    assert st_a == st_b and st_a["matches"] > 0
    # a read after asynchronous steps waits for them
    a.step(5)
    b.step_async(5)
    _same(b.state(), a.state(), S.PREC_FP32_FP64NC, f"{dim}D read")
    b.sync()
    a.close()
    b.close()


def test_pool_async_steps_equal_synchronous_steps():
    prec = S.PREC_FP32_FP64NC
    x = _system(5000, 3, 31, 1000.0, prec, kappa=0.2, replica=1)
    y = _system(4000, 3, 32, 1000.0, prec, kappa=0.7, replica=2)
    p, q = _pool(SHARED3, prec, slot_cap=9500), _pool(SHARED3, prec, slot_cap=9500)
    px, qx = p.admit(**x), q.admit(**x)
    p.step(6)
    q.step_async(6)
    py, qy = p.admit(**y), q.admit(**y)  # admission is ordered after the enqueued steps
    p.step(9)
    q.step_async(4)
    q.step_async(5)
    q.sync()
    _same(q.member_state(qx), p.member_state(px), prec, "member x")
    _same(q.member_state(qy), p.member_state(py), prec, "member y")
    p.close()
    q.close()


def test_logging_and_timing_handles_refuse_async_steps():
    for kw in (dict(debug=True, debug_cap=1 << 16), dict(timing=True)):
        h = _handle(3, **kw)
        with pytest.raises(S.SimError) as e:
            h.step_async(1)
        assert e.value.code == S.SIM_EINVAL
        h.step(1)  # the synchronous form still runs
        h.sync()
        h.close()
