"""Seeded synthetic inputs shared by the HIP path's callers and the oracle's tests.

This module only places particles: uniform positions in a periodic box with the
A:B mix of the workload and no initial A-B overlap.  It contains none of the
method's arithmetic (no displacement, no Green's function, no random draw of the
step itself), so both sides can take their initial state from here.

Workloads (all periodic, uniform, A:B = 1:1, no C at t = 0):

* ``cfg_abs3d``      3D irreversible A+B->C, absorbing; 1,000 A + 1,000 B, L = 1 um,
                     D = 1 um^2/s, sigma = 5 nm, dt = 1 us, FP64.
* ``cfg_rad3d``      3D reversible A+B<->C, radiation; 5e5 A + 5e5 B, L = 10 um,
                     D = 1 um^2/s, sigma = 5 nm, kappa = 0.1 um^3/s, k_off = 10/s, dt = 10 us,
                     binary32 displacements and state, binary64 near-contact pair arithmetic.
                     ``cfg_rad3d_dense`` is the heaviest pair load of the same grid
                     (D = 10 um^2/s, sigma = 10 nm).
* ``cfg_mem2d``      2D membrane A+B<->C; 5e5 A + 5e5 B on L = 20 um, D = 0.1 um^2/s,
                     sigma = 5 nm, kappa_2D = 0.05 um^2/s, k_off = 10/s, dt = 100 us.
                     ``cfg_mem2d_small_tau`` is the same with dt = 5 us (tau = 0.04).
"""
from __future__ import annotations

import numpy as np

SP_A, SP_B, SP_C, SP_FREE, SP_RESERVED = 0, 1, 2, 3, 4
BC_ABS, BC_REF, BC_RAD = 0, 1, 2
PREC_FP64, PREC_FP32, PREC_FP32_FP64NC, PREC_FP32D_FP64NC = 0, 1, 2, 3


def workload(name: str, **over) -> dict:
    """Parameter set of a named workload (units: um, s)."""
    base = {
        "cfg_abs3d": dict(dim=3, bc=BC_ABS, n_a=1000, n_b=1000, box=1.0, D=(1.0, 1.0), sigma=0.005,
                          kappa_a=0.0, k_off=0.0, dt=1e-6, steps=100, precision=PREC_FP64),
        "cfg_rad3d": dict(dim=3, bc=BC_RAD, n_a=500_000, n_b=500_000, box=10.0, D=(1.0, 1.0), sigma=0.005,
                          kappa_a=0.1, k_off=10.0, dt=1e-5, steps=1000, precision=PREC_FP32D_FP64NC),
        "cfg_rad3d_dense": dict(dim=3, bc=BC_RAD, n_a=500_000, n_b=500_000, box=10.0, D=(10.0, 10.0),
                                sigma=0.010, kappa_a=0.1, k_off=10.0, dt=1e-5, steps=1000,
                                precision=PREC_FP32D_FP64NC),
        "cfg_mem2d": dict(dim=2, bc=BC_RAD, n_a=500_000, n_b=500_000, box=20.0, D=(0.1, 0.1), sigma=0.005,
                          kappa_a=0.05, k_off=10.0, dt=1e-4, steps=1000, precision=PREC_FP32_FP64NC),
        "cfg_mem2d_small_tau": dict(dim=2, bc=BC_RAD, n_a=500_000, n_b=500_000, box=20.0, D=(0.1, 0.1),
                                    sigma=0.005, kappa_a=0.05, k_off=10.0, dt=5e-6, steps=1000,
                                    precision=PREC_FP32_FP64NC),
    }[name]
    cfg = dict(base)
    cfg.update(over)
    D = tuple(cfg["D"])
    if len(D) == 2:  # D_C defaults to D_A D_B / (D_A + D_B)
        D = (D[0], D[1], D[0] * D[1] / (D[0] + D[1]))
    cfg["D"] = D
    cfg["name"] = name
    return cfg


def _round(pos: np.ndarray, box: float, f32: bool) -> np.ndarray:
    if f32:
        pos = pos.astype(np.float32).astype(np.float64)
        pos[pos >= box] -= box
    return pos


def uniform_state(n_a: int, n_b: int, *, box: float, dim: int, sigma: float, seed: int = 0,
                  f32: bool = True, max_rounds: int = 100):
    """Uniform A and B positions; every B closer than ``sigma`` to an A is redrawn.

    Returns ``(species, pos, n_redrawn)``: int32 species codes (A first, then B),
    float64 positions of shape (n, dim) that are exactly representable in binary32
    when ``f32``, and how many B positions were redrawn.
    """
    from scipy.spatial import cKDTree

    rng = np.random.Generator(np.random.PCG64(seed))
    n = n_a + n_b
    pos = _round(rng.random((n, dim)) * box, box, f32)
    species = np.concatenate([np.full(n_a, SP_A, np.int32), np.full(n_b, SP_B, np.int32)])
    redrawn = 0
    if n_a and n_b:
        tree = cKDTree(pos[:n_a], boxsize=box)
        todo = np.arange(n_a, n)
        for _ in range(max_rounds):
            d, _ = tree.query(pos[todo], k=1, distance_upper_bound=sigma)
            bad = todo[d < sigma]
            if bad.size == 0:
                break
            redrawn += int(bad.size)
            pos[bad] = _round(rng.random((bad.size, dim)) * box, box, f32)
            todo = bad
        else:
            raise RuntimeError("could not place B particles without overlap")
    return species, pos, redrawn


def state_for(cfg: dict, seed: int = 0, scale: float = 1.0):
    """Initial state of a workload; ``scale`` shrinks the particle count and the box
    volume together so the density stays that of the workload."""
    n_a = max(1, int(round(cfg["n_a"] * scale)))
    n_b = max(1, int(round(cfg["n_b"] * scale)))
    f32 = cfg["precision"] != PREC_FP64
    box = cfg["box"] * scale ** (1.0 / cfg["dim"])
    if f32:  # a binary32 state needs a binary32 box edge
        box = float(np.float32(box))
    sp, pos, red = uniform_state(n_a, n_b, box=box, dim=cfg["dim"], sigma=cfg["sigma"], seed=seed, f32=f32)
    return sp, pos, box, red


def ensemble(n_rep: int = 4096, seed: int = 0, n_min: float = 1e3, n_max: float = 1e5, f32: bool = True):
    """Replicas of the batched 3D workload: particle counts log-uniform in [n_min, n_max] and
    kappa_a uniform in [0.01, 1] um^3/s, both drawn from PCG64(seed); half A, half B, uniform in
    a periodic cube of edge (N/1000)^(1/3) um (rounded to binary32), every B closer than 5 nm
    to an A redrawn; replica r is seeded 1000 + r and keyed r."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.exp(rng.uniform(np.log(n_min), np.log(n_max), n_rep)).astype(np.int64)
    kappas = rng.uniform(0.01, 1.0, n_rep)
    reps = []
    for r in range(n_rep):
        n = int(counts[r])
        box = float(np.float32((n / 1000.0) ** (1.0 / 3.0)))
        sp, pos, _ = uniform_state(n // 2, n - n // 2, box=box, dim=3, sigma=0.005, seed=1000 + r, f32=f32)
        reps.append(dict(species=sp, pos=pos, box=box, kappa=float(kappas[r]), replica=r))
    return reps


def lattice_targets(m: int, spacing: float, n_b: int, sigma: float, seed: int = 0):
    """m^3 targets (species 0) at ((i, j, k) + 1/4) * spacing and n_b B's (species 1) uniform in
    the periodic box of edge m * spacing, each B closer than sigma to a target redrawn."""
    L = m * spacing
    g = (np.arange(m) + 0.25) * spacing
    a = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.Generator(np.random.PCG64(seed))
    b = rng.random((n_b, 3)) * L
    for _ in range(100):
        d = b - (np.floor(b / spacing - 0.25 + 0.5) + 0.25) * spacing  # to the nearest lattice point
        bad = np.flatnonzero(np.sum(d * d, axis=1) < sigma * sigma)
        if bad.size == 0:
            break
        b[bad] = rng.random((bad.size, 3)) * L
    b = b.astype(np.float32).astype(np.float64)
    b[b >= L] = 0.0
    sp = np.concatenate([np.zeros(len(a), np.int32), np.ones(n_b, np.int32)])
    return sp, np.concatenate([a, b]), L
