"""The autotuner's choices change only the speed: every candidate cell edge, pair-search kernel
and launch shape gives the same trajectory, bit for bit."""
import numpy as np
import pytest

from paper_1107_0270_amd import autotune as AT
from paper_1107_0270_amd import inputs as I
from paper_1107_0270_amd import sim as S

pytestmark = pytest.mark.gpu

CASES = {
    "rad3d": dict(dim=3, dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, bc=S.BC_RADIATION, kappa=0.1, k_off=2000.0,
                  density=1000.0, n=30000, prec=S.PREC_FP32_FP64NC),
    "rad3d_dense_fp64": dict(dim=3, dt=1e-5, D=(10.0, 10.0, 5.0), sigma=0.01, bc=S.BC_RADIATION, kappa=1.0,
                             k_off=2000.0, density=8000.0, n=20000, prec=S.PREC_FP64),
    "mem2d": dict(dim=2, dt=5e-6, D=(0.1, 0.1, 0.05), sigma=0.005, bc=S.BC_RADIATION, kappa=0.05, k_off=2000.0,
                  density=2500.0, n=20000, prec=S.PREC_FP32_FP64NC),
}


@pytest.mark.parametrize("name", list(CASES))
def test_every_candidate_gives_the_same_trajectory(name):
    c = dict(CASES[name])
    dim, n, prec, density = c.pop("dim"), c.pop("n"), c.pop("prec"), c.pop("density")
    box = float(np.float32((n / density) ** (1.0 / dim)))
    sp, pos, _ = I.uniform_state(n // 2, n - n // 2, box=box, dim=dim, sigma=c["sigma"], seed=8, f32=prec != S.PREC_FP64)

    def make(cell, ps, **launch):
        return S.Sim(dim=dim, box=box, species=sp, pos=pos, precision=prec, seed=2, cell=cell, pair_search=ps,
                     **launch, **c)

    ref = make(0.0, S.PAIRS_AUTO)
    rcut, cell0 = ref.derived()["rcut"], ref.derived()["cell"]
    ref.step(12)
    want = ref.state()
    want_stats = ref.stats(total=True)
    ref.close()
    seen = set()
    # every cell/search candidate at the default launch shapes, then the default grid at launch
    # shapes from one workgroup per XCD to far more workgroups than pairs or events
    shapes = [(cell, ps, {}) for cell, ps in AT.candidates(box, dim, rcut, cell0)]
    shapes += [(0.0, S.PAIRS_AUTO, dict(pair_blocks=pb, event_blocks=eb)) for pb, eb in ((8, 1), (200, 77), (4096, 4096))]
    for cell, ps, launch in shapes:
        sim = make(cell, ps, **launch)
        g = tuple(sim.grid())
        sim.step(12)
        got = sim.state()
        st = sim.stats(total=True)
        sim.close()
        seen.add(g)
        assert np.array_equal(got[0], want[0]), (cell, ps, g, launch)
        live = want[0] <= S.SP_C
        assert np.array_equal(got[1][live], want[1][live]), (cell, ps, g, launch)
        cc = want[0] == S.SP_C
        assert np.array_equal(got[2][cc], want[2][cc]), (cell, ps, g, launch)
        for k in ("pairs", "cand", "matches", "react", "decay", "geminate"):
            assert st[k] == want_stats[k], (k, cell, ps, g, launch)
    assert len(seen) >= 4  # several grids and both kernels were exercised
    assert want_stats["react"] > 0


def test_tune_returns_a_timed_choice():
    n, box = 20000, float(np.float32((20000 / 1000.0) ** (1 / 3)))
    sp, pos, _ = I.uniform_state(n // 2, n - n // 2, box=box, dim=3, sigma=0.005, seed=1, f32=True)
    kw = dict(dim=3, dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, bc=S.BC_RADIATION, kappa=0.1, k_off=10.0)
    probe = S.Sim(box=box, species=sp, pos=pos, **kw)
    rcut = probe.derived()["rcut"]
    probe.close()
    best, table = AT.tune(lambda cell, ps, **launch: S.Sim(box=box, species=sp, pos=pos, cell=cell, pair_search=ps,
                                                           **launch, **kw),
                          box=box, dim=3, rcut=rcut, steps=5, warmup=2, pair_blocks=(256, 2048), event_blocks=(512,))
    keys = ("cell", "pair_search", "pair_blocks", "event_blocks")
    fastest = min(table, key=lambda r: r["ms_per_step"])
    assert {k: fastest[k] for k in keys} == best
    assert sum(1 for r in table if r["pair_blocks"] or r["event_blocks"]) == 3  # stage 2 timed each launch shape
