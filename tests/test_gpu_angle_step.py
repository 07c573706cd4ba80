"""The step's angle stage (Sec. 3, Details; eqs. genericGF3D and genericGF) and sim_eval_angle
run the same one-workgroup draw: on the radii R'', R0 and the uniform the step used for each
propagated pair, sim_eval_angle must return the step's angle bit for bit.  This pins the
stage's inputs (the clamped pre-step radius, the counter-based uniform of {slot A, slot B,
step, ANG}) and its use of the draw, on pairs of one to six batches of 128 quadrature nodes.
3D: every propagated pair, bit for bit.  2D: the log holds cos theta, computed on the GPU from
the drawn |theta|, so the comparison takes numpy's cosine of sim_eval_angle's |theta| and allows
it two units in the last place."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1107_0270_amd import inputs as I
from paper_1107_0270_amd import sim as S

pytestmark = pytest.mark.gpu

TAG_ANG = 13


def _u(w):
    return (np.asarray(w, np.float64) + 0.5) * 2.0 ** -32


def _batches(dim, R, R0, tau):
    """Node batches of 128 of the pair's quadrature (the kernel's layout: 16-point panels to
    sqrt(40 / tau), in 2D twelve geometric ones on [4^-12, 1] first)."""
    R, R0 = max(R, 1.0), max(R0, 1.0)
    X = math.sqrt(40.0 / tau)
    hmax = min(1.0, 2.0 * math.pi / (R + R0 - 1.0))
    if dim == 3:
        q = 16 * math.ceil(X / hmax)
    else:
        x1 = min(X, 1.0)
        q = 16 * (12 + (math.ceil((X - x1) / hmax) if X > x1 else 0))
    return -(-q // 128)


def _propagated(gpu, step=0, key=(0, 0)):
    gp, gm = gpu.dbg_pairs(), gpu.dbg_matches()
    R0_of = {(int(r["i"]), int(r["j"])): float(r["R0"]) for r in gp}
    prop = gm[gm["reacted"] == 0]
    R0 = np.array([max(R0_of[(int(r["i"]), int(r["j"]))], 1.0) for r in prop])
    u = np.array([_u(O.philox((int(r["i"]), int(r["j"]), step, TAG_ANG), key)[0]) for r in prop])
    return prop, prop["Rpp"].astype(np.float64), R0, u


@pytest.mark.parametrize("dt", [6.25e-6, 1e-5])
def test_3d_step_angles_equal_eval_angle(dt):
    # the 3D radiation workload at 4.2e5 particles in a 7.5 um box (about the same density);
    # tau = 0.5 puts every pair in two batches or more, tau = 0.8 (the benchmark's) only
    # pairs with R + R0 > 8.1
    cfg = I.workload("cfg_rad3d", n_a=210_000, n_b=210_000, box=7.5, dt=dt)
    sp, pos, _ = I.uniform_state(cfg["n_a"], cfg["n_b"], box=cfg["box"], dim=3, sigma=cfg["sigma"], seed=2)
    gpu = S.Sim(dim=3, box=cfg["box"], dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"], bc=cfg["bc"],
                kappa=cfg["kappa_a"], k_off=cfg["k_off"], precision=cfg["precision"], species=sp, pos=pos,
                debug=True, debug_cap=1 << 20)
    tau = gpu.derived()["tau"]
    gpu.step()
    prop, Rpp, R0, u = _propagated(gpu)
    nb = np.array([_batches(3, a, b, tau) for a, b in zip(Rpp, R0)])
    print("tau", tau, "propagated", len(prop), "by batches", np.bincount(nb))
    assert len(prop) >= 50
    assert np.count_nonzero(nb >= 2) >= (len(prop) // 2 if tau < 0.6 else 0)
    c = gpu.eval_angle(Rpp, R0, u)
    got = prop["cos_theta"].astype(np.float64)
    bad = np.flatnonzero(c.view(np.uint64) != got.view(np.uint64))
    assert bad.size == 0, [(Rpp[k], R0[k], u[k], c[k], got[k], nb[k]) for k in bad[:5]]
    gpu.close()


def test_2d_step_angles_equal_eval_angle():
    # the membrane workload at full size (tau = 0.8: three batches a pair or more)
    cfg = I.workload("cfg_mem2d")
    sp, pos, _ = I.uniform_state(cfg["n_a"], cfg["n_b"], box=cfg["box"], dim=2, sigma=cfg["sigma"], seed=0)
    gpu = S.Sim(dim=2, box=cfg["box"], dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"], bc=cfg["bc"],
                kappa=cfg["kappa_a"], k_off=cfg["k_off"], precision=cfg["precision"], species=sp, pos=pos,
                green2d=S.G2_EXACT, eps_cut=1e-6, debug=True, debug_cap=1 << 22)
    tau = gpu.derived()["tau"]
    gpu.step()
    prop, Rpp, R0, u = _propagated(gpu)
    nb = np.array([_batches(2, a, b, tau) for a, b in zip(Rpp, R0)])
    print("tau", tau, "propagated", len(prop), "by batches", np.bincount(nb))
    assert np.count_nonzero(nb >= 3) >= 1000
    th = gpu.eval_angle(Rpp, R0, u)
    got = prop["cos_theta"].astype(np.float64)
    d = np.abs(np.cos(th) - got)
    k = int(np.argmax(d))
    assert d[k] <= 2.0 * np.spacing(1.0), (Rpp[k], R0[k], u[k], th[k], got[k], nb[k])
    gpu.close()
