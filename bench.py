#!/usr/bin/env python3
"""Throughput of the coarse-grained Green's-function BD step on one MI355X.

Workload (synthetic, seeded): 3D reversible A + B <-> C with a radiation surface,
5e5 A + 5e5 B uniform in a periodic 10 um cube, D_A = D_B = 1 um^2/s, sigma = 5 nm,
kappa_a = 0.1 um^3/s, k_off = 10/s, dt = 10 us, binary32 state with binary64
near-contact arguments.  One step = move, bin, pairs + p_enc, selection,
propagation/reaction, dissociation (the whole step of Sec. 3).

Prints one JSON line.  Kernel durations come from HIP events recorded on the
library's stream around every kernel of the timed steps.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(kernel, n_live, n_a, n_b, n_keys, rec_bytes):
    """HBM bytes one launch of a stage must move at least (each datum once)."""
    return {
        "move": (2 * rec_bytes + 4) * n_live + 8 * n_keys,      # read record, write moved record + rank, count buckets
        "scan": 12 * n_keys,                                     # read counts, write starts, clear counts
        "scatter": (2 * rec_bytes + 8) * n_live,                 # read moved record + rank + start, write record
        "pairs": rec_bytes * (n_a + n_b) + 4 * n_keys // 3,      # A and B records once, B bucket starts
    }.get(kernel)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=20, help="oracle steps timed for the CPU baseline (0 = skip)")
    ap.add_argument("--no-timing", action="store_true", help="time without per-kernel events")
    ap.add_argument("--pair-search", choices=["auto", "bricks", "direct"], default="auto",
                    help="pair-search kernel (auto = the library's choice)")
    ap.add_argument("--cell", type=float, default=0.0, help="cell edge in um (0 = the library's choice)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not supported", "n_gpus": args.gpus}))
        sys.exit(2)

    from paper_1107_0270_amd import inputs as I
    from paper_1107_0270_amd import sim as S

    cfg = I.workload("cfg_rad3d")
    t0 = time.time()
    sp, pos, box, red = I.state_for(cfg, seed=0)
    log(f"[bench] state: {len(sp)} particles, {red} redrawn overlaps, {time.time() - t0:.1f}s")
    def make(timing):
        return S.Sim(dim=3, box=box, dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"], bc=cfg["bc"], kappa=cfg["kappa_a"],
                     k_off=cfg["k_off"], precision=cfg["precision"], seed=0, species=sp, pos=pos, timing=timing, cell=args.cell,
                     pair_search={"auto": S.PAIRS_AUTO, "bricks": S.PAIRS_BRICKS, "direct": S.PAIRS_DIRECT}[args.pair_search])

    def timed(sim):
        sim.step(args.warmup)
        sim.kernel_times()  # drop warm-up timings
        c0, s0 = sim.counts(), sim.stats(total=True)
        t0 = time.perf_counter()
        sim.step(args.steps)  # returns after a stream synchronisation
        el = time.perf_counter() - t0
        c1, s1 = sim.counts(), sim.stats(total=True)
        n_live = 0.5 * ((c0["A"] + c0["B"] + c0["C"]) + (c1["A"] + c1["B"] + c1["C"]))
        return el, n_live, s1["pairs"] - s0["pairs"], c0, c1, sim.kernel_times()

    # pass 1: the step as one HIP graph replay (no per-kernel events) -> value
    sim = make(False)
    der, grid = sim.derived(), sim.grid()
    log(f"[bench] derived {der} grid {grid}")
    el, n_live, pairs, c0, c1, _ = timed(sim)
    sim.close()
    ps = n_live * args.steps / el
    log(f"[bench] graph: {args.steps} steps in {el * 1e3:.1f} ms; {ps:.3e} particle-steps/s; {pairs / el:.3e} pair evals/s")
    # pass 2: the same steps with HIP events around every kernel -> kernel durations
    kt, el_ev = {}, None
    if not args.no_timing:
        sim = make(True)
        el_ev, _, _, c0, c1, kt = timed(sim)
        sim.close()
        log(f"[bench] events: {args.steps} steps in {el_ev * 1e3:.1f} ms; kernel times {kt}")

    # dominant kernel and its roofline
    rec_bytes = 16
    n_keys = 3 * grid[3]
    per = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kt.items()}
    tot = {k: v[0] for k, v in kt.items()}
    dom = max(tot, key=tot.get) if any(tot.values()) else None
    roof = None
    if dom is not None and per[dom] > 0:
        nb = algorithmic_bytes(dom, n_live, 0.5 * (c0["A"] + c1["A"]), 0.5 * (c0["B"] + c1["B"]), n_keys, rec_bytes)
        if nb is not None:
            ach = nb / (per[dom] * 1e-3) / 1e9
            roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "bytes_per_launch": int(nb),
                    "avg_launch_ms": round(per[dom], 5)}

    cpu = None
    if args.cpu_steps > 0:
        import oracle as O

        orc = O.OracleSim(dim=3, bc=cfg["bc"], box=[box] * 3, dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"],
                          kappa_a=cfg["kappa_a"], k_off=cfg["k_off"], store_f32=True, species=sp, pos=pos)
        tc = time.perf_counter()
        orc.step(args.cpu_steps)
        tc = time.perf_counter() - tc
        cpu = {"value": round(len(sp) * args.cpu_steps / tc, 1), "unit": "particle-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{args.cpu_steps} steps of the same 1e6-particle workload from the same initial state, "
                         f"single-threaded FP64 C oracle ({tc:.1f} s)"}
        log(f"[bench] cpu baseline {cpu}")

    out = {
        "metric": "particle-steps/s at 1e-6 pair-probability accuracy",
        "value": round(ps, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el * 1e3 / args.steps, 5),
        "ms_per_step_with_kernel_events": None if el_ev is None else round(el_ev * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "pair_evals_per_s": round(pairs / el, 1),
        "config": {"workload": "3D reversible A+B<->C, radiation surface: 5e5 A + 5e5 B, periodic L=10 um, "
                               "D=1 um^2/s, sigma=5 nm, kappa=0.1 um^3/s, k_off=10/s, dt=10 us",
                   "precision": "binary32 state and p_enc, binary64 near-contact arguments and propagation",
                   "particles": len(sp), "r_cut_um": der["rcut"], "cells": grid[:3],
                   "pair_search": {S.PAIRS_BRICKS: "lds-bricks", S.PAIRS_DIRECT: "direct"}[grid[4]],
                   "step_launch": "one hipGraph replay per step"},
        "roofline": roof,
        "kernel_ms_per_step": {k: round(v[0] / max(args.steps, 1), 5) for k, v in kt.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
