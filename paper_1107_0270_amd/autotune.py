"""Autotuner for the run-time choices of a step: the cell edge of the cell list, the
pair-search kernel (direct neighbour-bucket search or LDS bricks) and the launch shapes of the
pair stage and of the event kernel (workgroups per launch).

The choices change only how fast a step runs, never what it computes: whatever the grid, the
pair list is the set of all A-B pairs within r_cut, every choice among candidates goes by
slot, and the pair-stage and event kernels stride over their work whatever their grid.  So the
tuner times candidates on the caller's own state and keeps the fastest.

Usage:
    best, table = tune(lambda cell, pair_search, **launch: Sim(..., cell=cell, pair_search=pair_search, **launch),
                       box=..., dim=..., rcut=...)
    sim = Sim(..., **best)

A TuneCache keeps the choice per workload signature (dimension, precision, boundary, and the
binned particle density, tau and count) in a JSON file, so a workload is tuned once.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import sim as S

# cell edges tried: multiples of r_cut (the smallest edge the library takes) and of the library's
# own choice (about one B per cell), which is used as it stands too
CELL_FACTORS = (1.0, 1.25, 1.5, 2.0, 3.0)
DEFAULT_FACTORS = (0.6, 0.75, 0.9, 1.15, 1.35, 1.6, 2.0)
SEARCHES = (S.PAIRS_DIRECT, S.PAIRS_BRICKS)
# workgroups per launch tried for the pair-evaluation/selection kernels and for the event kernel
# (the library's default is 1024 for both)
PAIR_BLOCKS = (256, 512, 1024, 2048)
EVENT_BLOCKS = (256, 512, 1024, 2048)


def grid_of(box, dim, cell, rcut):
    """Cells per axis for a requested cell edge (the library's rule: edge >= r_cut, at most
    2048 cells per axis, fewer than three cells on an axis means one)."""
    c = max(cell, rcut)
    out = []
    for k in range(dim):
        L = box[k] if hasattr(box, "__len__") else box
        m = min(int(math.floor(L / c)), 2048)
        out.append(m if m >= 3 else 1)
    return tuple(out)


def candidates(box, dim, rcut, cell0=None, factors=CELL_FACTORS, default_factors=DEFAULT_FACTORS,
               searches=SEARCHES):
    """(cell, pair_search) pairs to time: the library's default (cell 0), then each multiple of
    r_cut and of the default edge cell0 that is at least r_cut and gives a distinct grid, each
    with every search kernel."""
    seen, out = set(), []
    edges = [f * rcut for f in factors]
    if cell0:
        seen.add(grid_of(box, dim, cell0, rcut))
        edges += [f * cell0 for f in default_factors]
    for cell in [0.0] + sorted(e for e in edges if e >= rcut):
        g = grid_of(box, dim, cell, rcut) if cell > 0 else None
        if g is not None and g in seen:
            continue
        if g is not None:
            seen.add(g)
        for ps in searches:
            out.append((cell, ps))
    return out


def time_steps(sim, steps, warmup, repeats=2):
    """Best wall time per step over `repeats` runs of `steps` graph-replayed steps (sim_step
    returns when its steps are done)."""
    sim.step(warmup)
    best = float("inf")
    for _ in range(repeats):
        t0 = time.perf_counter()
        sim.step(steps)
        best = min(best, (time.perf_counter() - t0) / steps)
    return best


def tune(make, *, box, dim, rcut, cell0=None, steps=30, warmup=10, factors=CELL_FACTORS,
         default_factors=DEFAULT_FACTORS, searches=SEARCHES, pair_blocks=PAIR_BLOCKS, event_blocks=EVENT_BLOCKS,
         log=None):
    """Time every candidate; returns (choice, table) with choice = {'cell', 'pair_search',
    'pair_blocks', 'event_blocks'}.  `make(cell, pair_search, **launch)` returns a fresh handle on
    the workload's initial state (launch: pair_blocks and event_blocks, absent = the library's
    default); cell0 is the edge the library picks by itself (sim.derived()['cell']).

    Stage 1 times every (cell, pair_search) candidate at the default launch shapes, skipping
    those for which the library picks a kernel and grid already timed.  Stage 2 then times, on
    the best of stage 1, each pair-stage workgroup count and, on the best of those, each event
    workgroup count (empty tuples skip stage 2)."""
    table, done = [], set()

    def timed(cell, ps, **launch):
        sim = make(cell, ps, **launch)
        try:
            g = tuple(int(x) for x in sim.grid())
            if not launch:
                if g in done:
                    return None
                done.add(g)
            t = time_steps(sim, steps, warmup)
        finally:
            sim.close()
        row = {"cell": cell, "pair_search": ps, "grid": list(g[:3]), "kernel": "bricks" if g[4] == S.PAIRS_BRICKS
               else "direct", "pair_blocks": launch.get("pair_blocks", 0), "event_blocks": launch.get("event_blocks", 0),
               "ms_per_step": t * 1e3}
        table.append(row)
        if log:
            log(f"[autotune] cell {cell:.5f} ({'x'.join(map(str, g[:dim]))}) {row['kernel']} pair_blocks "
                f"{row['pair_blocks'] or 'default'} event_blocks {row['event_blocks'] or 'default'}: {t * 1e3:.4f} ms/step")
        return row

    for cell, ps in candidates(box, dim, rcut, cell0, factors, default_factors, searches):
        try:
            timed(cell, ps)
        except S.SimError as e:  # a grid the library does not take for this state (e.g. a brick too large)
            if e.code != S.SIM_EUNSUPPORTED:
                raise
    best = min(table, key=lambda r: r["ms_per_step"])
    choice = {"cell": best["cell"], "pair_search": best["pair_search"], "pair_blocks": 0, "event_blocks": 0}
    for key, values in (("pair_blocks", pair_blocks), ("event_blocks", event_blocks)):
        for v in values:
            row = timed(choice["cell"], choice["pair_search"], **dict(
                {k: choice[k] for k in ("pair_blocks", "event_blocks") if choice[k]}, **{key: v}))
            if row["ms_per_step"] < best["ms_per_step"]:
                best = row
                choice[key] = v
    return choice, table


def signature(*, dim, precision, bc, n, box, tau):
    """Workload key: dimension, precision, boundary, and log2 bins of the particle density,
    of tau and of the particle count."""
    vol = 1.0
    for k in range(dim):
        vol *= box[k] if hasattr(box, "__len__") else box
    return "d{}-p{}-bc{}-rho{}-tau{}-n{}".format(dim, precision, bc, round(2 * math.log2(n / vol)),
                                                  round(2 * math.log2(tau)), round(math.log2(n)))


class TuneCache:
    """Choices per workload signature, kept in a JSON file."""

    def __init__(self, path):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def get(self, key):
        return self.data.get(key)

    def put(self, key, choice):
        self.data[key] = choice
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
