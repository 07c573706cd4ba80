"""A pool sized for its capacity (2^23 slots and 2^22 + 4,096 cells: 1.3e7 bucket keys, 3,073
scan tiles) has most of its keys in the unused tail of each species block, and the bucket scan
skips those tiles (their counts are zero and no kernel reads their offsets).  The cell lists
of Sec. 3 must come out exact all the same: members admitted at different steps, one of them
after another left, step bit for bit as they step alone on handles of their own size (whose
scans skip nothing), through the C-ABI."""
import pytest

from paper_1107_0270_amd import sim as S

from .test_gpu_pool import SHARED3, _pool, _same, _system

pytestmark = pytest.mark.gpu


def _alone(x, prec):
    sh = dict(SHARED3)
    sh.pop("dim")
    return S.Sim(dim=3, precision=prec, **sh, **x)


def test_members_of_a_large_pool_step_as_alone():
    prec = S.PREC_FP32_FP64NC
    x = _system(6000, 3, 41, 1000.0, prec, kappa=0.5, replica=3)
    y = _system(3000, 3, 42, 1000.0, prec, kappa=0.2, replica=4)
    z = _system(2000, 3, 43, 1000.0, prec, kappa=0.8, replica=5)
    pool = _pool(SHARED3, prec, slot_cap=1 << 23, cell_cap=(1 << 22) + 4096)
    ax = _alone(x, prec)
    mx = pool.admit(**x)
    pool.step(5)
    ax.step(5)
    ay = _alone(y, prec)
    my = pool.admit(**y)  # the high-water mark rises
    pool.step(5)
    ax.step(5)
    ay.step(5)
    _same(pool.member_state(mx), ax.state(), prec, "x")
    _same(pool.member_state(my), ay.state(), prec, "y")
    pool.retire(mx)
    az = _alone(z, prec)
    mz = pool.admit(**z)  # first fit: the cells x left
    pool.step(6)
    ay.step(6)
    az.step(6)
    _same(pool.member_state(my), ay.state(), prec, "y after x left")
    _same(pool.member_state(mz), az.state(), prec, "z in x's cells")
    st = ay.stats(total=True)
    assert st["matches"] > 0
    for h in (pool, ax, ay, az):
        h.close()
