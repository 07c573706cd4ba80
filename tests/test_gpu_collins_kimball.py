"""The GPU step at scale against the Collins-Kimball law: 79,507 static targets among 10^7
independent B's (1,000 per um^3), irreversible radiation reaction.  A target's survival is
exp(-rho_B int_0^t k(s) ds) with the time-dependent Collins-Kimball rate, an exact result for
independent B's; the targets sit 0.5 um apart, three diffusion lengths of the run, and the B's
lost to them are 0.15% of all.  A property that holds at any size."""
import numpy as np
import pytest

from paper_1107_0270_amd import inputs as I
from paper_1107_0270_amd import sim as S
from tests.ck_law import ck_survival

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kappa", [0.1, 1.0])
def test_static_targets_follow_collins_kimball(kappa):
    D, sigma, dt = 1.0, 0.005, 1e-5
    m, spacing = 43, 0.5
    L = m * spacing  # 21.5 um, exact in binary32
    n_b = int(round(1000.0 * L ** 3))
    sp, pos, L = I.lattice_targets(m, spacing, n_b, sigma, seed=11)
    sim = S.Sim(dim=3, box=L, dt=dt, D=(0.0, D, 0.5), sigma=sigma, bc=S.BC_RADIATION, kappa=kappa, k_off=0.0,
                eps_cut=1e-6, seed=5, species=sp, pos=pos)
    n_t = m ** 3
    done = 0
    for n in (100, 250, 500):
        sim.step(n - done)
        done = n
        got = sim.counts()["A"] / n_t
        want = ck_survival(n * dt, n_b / L ** 3, D, sigma, kappa)
        err = np.sqrt(want * (1 - want) / n_t)
        print(f"kappa {kappa}, {n} steps: survival {got:.5f}, Collins-Kimball {want:.5f} +- {err:.5f}")
        assert abs(got - want) < 4 * err
    sim.close()
