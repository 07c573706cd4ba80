"""The GPU step at scale against the equilibrium constant of A + B <-> C: a property that
holds at any size.  With a radiation surface of intrinsic rate kappa_a and dissociation into
a contact pair at rate k_off, detailed balance gives K = [C] / ([A][B]) = kappa_a / k_off; a
dilute mixture started from c0 free A and B per volume settles at the bound fraction
(c0 - y) / c0 with K y^2 + y - c0 = 0.  The runs take 10^5 particles, the pair cut-off at
eps = 1e-6, and relax for more than twenty relaxation times before averaging."""
import math

import numpy as np
import pytest

from paper_1107_0270_amd import inputs as I
from paper_1107_0270_amd import sim as S

pytestmark = pytest.mark.gpu


def _mass_action(K, c0):
    y = (-1.0 + math.sqrt(1.0 + 4.0 * K * c0)) / (2.0 * K)
    return (c0 - y) / c0


# diffusion-limited (kappa_a = 8 k_D) and reaction-limited (kappa_a = 0.8 k_D), both K = 0.01 um^3
@pytest.mark.parametrize("kappa,k_off", [(1.0, 100.0), (0.1, 10.0)])
def test_bound_fraction_follows_mass_action(kappa, k_off):
    n, dt = 100000, 1e-5
    box = float(np.float32((n / 1000.0) ** (1.0 / 3.0)))
    sp, pos, _ = I.uniform_state(n // 2, n - n // 2, box=box, dim=3, sigma=0.005, seed=3, f32=True)
    sim = S.Sim(dim=3, box=box, dt=dt, D=(1.0, 1.0, 0.5), sigma=0.005, bc=S.BC_RADIATION, kappa=kappa, k_off=k_off,
                eps_cut=1e-6, seed=7, species=sp, pos=pos)
    want = _mass_action(kappa / k_off, (n // 2) / box ** 3)
    sim.step(100000)
    fr = []
    for _ in range(50):
        sim.step(4000)
        fr.append(sim.counts()["C"] / (n // 2))
        assert sim.counts()["A"] + sim.counts()["C"] == n // 2  # conservation
    sim.close()
    fr = np.array(fr)
    err = fr.std() / math.sqrt(len(fr))  # samples 4,000 steps apart: about one relaxation time or more
    print(f"kappa {kappa} k_off {k_off}: bound fraction {fr.mean():.5f} +- {err:.5f}, mass action {want:.5f}")
    assert abs(fr.mean() - want) < max(4.0 * err, 1.5e-3)
