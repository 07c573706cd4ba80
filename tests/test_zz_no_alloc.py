"""The allocation-free entry point sim_eval_pairs_noalloc against sim_eval_pairs: the same p_enc
and p_reac, bit for bit, on two calls in a row, the second smaller and with other constants (its
2D expansion constants live in one array of the library that every call on a GPU rewrites)."""
import numpy as np
import pytest

from paper_1107_0270_amd import sim as S

pytestmark = pytest.mark.gpu


def _pairs(rng, n, rmax, tau):
    R = 1.0 + (rmax - 1.0) * rng.random(n)
    R0 = np.maximum(R + np.sqrt(2.0 * tau) * rng.standard_normal(n), 1.0)
    R[:3] = [0.9, 1.0, 1.0 + 1e-9]  # overlap, contact, just outside
    return R, R0


def _handle(cfg):
    sp = np.array([0, 1], np.int32)
    pos = np.array([[0.25] * cfg["dim"], [0.75] * cfg["dim"]])
    return S.Sim(box=1.0, species=sp, pos=pos, k_off=0.0, **cfg)


CASES = [
    # 2D membrane pairs (tau = 0.04), order 12 and a run-time order, two intrinsic rates
    (dict(dim=2, dt=5e-6, D=(0.1, 0.1, 0.05), sigma=0.005, bc=S.BC_RADIATION, kappa=0.05, precision=S.PREC_FP64),
     dict(dim=2, dt=4e-6, D=(0.1, 0.1, 0.05), sigma=0.005, bc=S.BC_RADIATION, kappa=0.5, precision=S.PREC_FP32_FP64NC,
          n_terms=10)),
    # 3D radiation pairs, the benchmark's precision and binary64
    (dict(dim=3, dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, bc=S.BC_RADIATION, kappa=0.1, precision=S.PREC_FP32_FP64NC),
     dict(dim=3, dt=1e-6, D=(1.0, 1.0, 0.5), sigma=0.005, bc=S.BC_RADIATION, kappa=1.0, precision=S.PREC_FP64)),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_pairs_match_the_handle(first, second):
    rng = np.random.default_rng(17)
    for cfg, n in ((first, 50000), (second, 7000)):  # the second call is smaller
        h = _handle(cfg)
        d = h.derived()
        R, R0 = _pairs(rng, n, d["rcut"] / d["a"], d["tau"])
        pe, pr = h.eval_pairs(R, R0)
        h.close()
        ge, gr = S.eval_pairs_noalloc(R, R0, **cfg)
        print(cfg["dim"], n, "max |dp_enc|", np.abs(ge - pe).max(), "max |dp_reac|", np.abs(gr - pr).max())
        assert np.array_equal(ge, pe) and np.array_equal(gr, pr)
