"""A 3D step that draws angles runs each event (Sec. 3, steps 2a-2c and the dissociations of
Sec. 2.2.5) and then the angle of its propagated pair (Sec. 3, Details) in one launch, a
workgroup per event.  When the step has more events than the launch has workgroups, each
workgroup takes its events first and then their angles.  The draws are keyed on the particles'
slots, not on the workgroups, so both forms must give the same step bit for bit: a handle
launched with few event workgroups (16 for a single system of about 34 events a step, 2 for a
batch of about 7) is compared with one launched with the default 1,024 (one event per
workgroup), for a single system at the density of the benchmark workload and for a batch of
replicas with frequent dissociations, through the C-ABI."""
import numpy as np
import pytest

from paper_1107_0270_amd import inputs as I
from paper_1107_0270_amd import sim as S

from .test_gpu_batch import SHARED, _replicas
from .test_gpu_pool import _same

pytestmark = pytest.mark.gpu


def _single(event_blocks, prec):
    # the 3D radiation workload at 6e4 particles in a 4 um box (about the benchmark's density)
    cfg = I.workload("cfg_rad3d", n_a=30_000, n_b=30_000, box=4.0)
    sp, pos, _ = I.uniform_state(cfg["n_a"], cfg["n_b"], box=cfg["box"], dim=3, sigma=cfg["sigma"], seed=9,
                                 f32=prec != S.PREC_FP64)
    return S.Sim(dim=3, box=cfg["box"], dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"], bc=cfg["bc"],
                 kappa=cfg["kappa_a"], k_off=cfg["k_off"], precision=prec, species=sp, pos=pos, event_blocks=event_blocks)


@pytest.mark.parametrize("prec", [S.PREC_FP32D_FP64NC, S.PREC_FP64])
def test_events_beyond_the_grid_give_the_same_step(prec):
    a, b = _single(0, prec), _single(16, prec)
    for k in range(3):
        a.step(5)
        b.step(5)
        _same(b.state(), a.state(), prec, f"after {5 * (k + 1)} steps")
    sa, sb = a.stats(total=True), b.stats(total=True)
    print("matches", sa["matches"], "per step", sa["matches"] / 15, "reactions", sa["react"], "decays", sa["decay"])
    assert sa == sb
    assert sa["matches"] / 15 > 16 and sa["react"] > 0
    a.close()
    b.close()


def test_batch_events_beyond_the_grid_give_the_same_step():
    prec = S.PREC_FP32_FP64NC
    reps = _replicas([600, 2200, 1000, 3400, 1500], prec)
    shared = dict(SHARED, k_off=20000.0)  # a C dissociates with probability 0.18 a step
    a = S.Sim.batch(reps, precision=prec, **shared)
    b = S.Sim.batch(reps, precision=prec, event_blocks=2, **shared)
    a.step(20)
    b.step(20)
    _same(b.state(), a.state(), prec, "batch")
    sa, sb = a.stats(total=True), b.stats(total=True)
    print("matches", sa["matches"], "reactions", sa["react"], "decays", sa["decay"])
    assert sa == sb and sa["matches"] > 2 * 20 and sa["decay"] > 0
    a.close()
    b.close()
