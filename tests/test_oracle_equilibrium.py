"""Pin of the oracle's reversible step against the equilibrium constant (CPU only).

For A + B <-> C with a radiation surface of intrinsic rate kappa_a (Sec. 2.2.3) and a
dissociation rate k_off into a contact pair (Sec. 2.2.5), detailed balance of the
two-body problem gives the equilibrium constant K = [C] / ([A][B]) = kappa_a / k_off,
whatever D and sigma.  In a dilute ideal mixture that started from c0 free A and B per
volume, the free concentration y solves K y^2 + y - c0 = 0 and the bound fraction is
(c0 - y) / c0.  The cut-off is taken at eps = 1e-6 (pairs whose reaction probability
within a step is below 1e-6 are left out), so the law of mass action holds to far below
the statistical error of these runs; the paper's 1e-3 cut-off leaves out a measurable
part of the association flux (about half a per cent in the reaction-limited case).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1107_0270_amd import inputs as I


def _mass_action(K, c0):
    y = (-1.0 + math.sqrt(1.0 + 4.0 * K * c0)) / (2.0 * K)
    return (c0 - y) / c0


# (kappa_a, k_off, relaxation steps): K = 0.01 and 0.002 um^3.  Near equilibrium the bound
# fraction relaxes at about k_off (1 - kappa/(kappa + k_D)) + 2 k_eff y, k_D = 4 pi sigma D_eff
# (the dissociations that escape geminate recombination, and the Collins-Kimball association):
# about 2,000 and 1,200 steps here; the runs relax ten times that long.
@pytest.mark.parametrize("kappa,k_off,relax", [(1.0, 100.0, 20000), (0.2, 100.0, 12000)])
def test_reversible_equilibrium_constant(kappa, k_off, relax):
    n, dt = 2000, 1e-5
    box = (n / 1000.0) ** (1.0 / 3.0)  # 500 A and 500 B per um^3
    want = _mass_action(kappa / k_off, (n // 2) / box ** 3)
    sp, pos, _ = I.uniform_state(n // 2, n - n // 2, box=box, dim=3, sigma=0.005, seed=3, f32=False)
    orc = O.OracleSim(dim=3, bc=O.BC_RAD, box=[box] * 3, dt=dt, D=(1.0, 1.0, 0.5), sigma=0.005, kappa_a=kappa,
                      k_off=k_off, eps_cut=1e-6, seed=5, species=sp, pos=pos)
    orc.step(relax)
    fr = []
    for _ in range(250):
        orc.step(100)
        s, _, _ = orc.state()
        fr.append(np.sum(s == O.SP_C) / (n // 2))
    fr = np.array(fr)
    # samples 100 steps apart are correlated over about twice the relaxation time
    err = fr.std() / math.sqrt(len(fr) * 100.0 / (2.0 * relax / 10.0))
    print(f"kappa {kappa} k_off {k_off}: bound fraction {fr.mean():.4f} +- {err:.4f}, mass action {want:.4f}")
    assert abs(fr.mean() - want) < 4.0 * err
