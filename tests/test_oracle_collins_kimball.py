"""Pin of the oracle's irreversible step against the Collins-Kimball law (CPU only).

Static targets A (D_A = 0) among B's diffusing independently with D_B react through a
radiation surface of intrinsic rate kappa_a at sigma.  A target's survival is then
exp(-rho_B int_0^t k(s) ds) with the time-dependent Collins-Kimball rate k(s), which starts at
kappa_a and settles at k_CK = 4 pi sigma D kappa_a / (4 pi sigma D + kappa_a): an exact result
of the two-body problem for independent B's.  The targets sit half a micrometre apart, three
diffusion lengths of the run, so they do not compete for B's; the B's lost to the targets are
0.1% of them.
"""
import numpy as np

import oracle as O
from paper_1107_0270_amd import inputs as I
from tests.ck_law import ck_survival


def test_static_targets_follow_collins_kimball():
    D, sigma, kappa, dt = 1.0, 0.005, 0.1, 1e-5
    m, spacing, n_b = 4, 0.5, 8000  # 64 targets in 8 um^3, 1,000 B per um^3
    checks = (100, 250, 500)
    alive = np.zeros(len(checks))
    n_t = 0
    for seed in range(8):
        sp, pos, L = I.lattice_targets(m, spacing, n_b, sigma, seed=seed)
        orc = O.OracleSim(dim=3, bc=O.BC_RAD, box=[L] * 3, dt=dt, D=(0.0, D, 0.5), sigma=sigma, kappa_a=kappa,
                          eps_cut=1e-6, seed=seed, species=sp, pos=pos)
        done = 0
        for c, n in enumerate(checks):
            orc.step(n - done)
            done = n
            s, _, _ = orc.state()
            alive[c] += np.sum(s == O.SP_A)
        n_t += m ** 3
    rho = n_b / L ** 3
    for c, n in enumerate(checks):
        want = ck_survival(n * dt, rho, D, sigma, kappa)
        got = alive[c] / n_t
        err = np.sqrt(want * (1 - want) / n_t)
        print(f"{n} steps: survival {got:.4f}, Collins-Kimball {want:.4f} +- {err:.4f}")
        assert abs(got - want) < 4 * err
