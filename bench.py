#!/usr/bin/env python3
"""Throughput of the coarse-grained Green's-function BD step on one MI355X.

Workload (synthetic, seeded): 3D reversible A + B <-> C with a radiation surface,
5e5 A + 5e5 B uniform in a periodic 10 um cube, D_A = D_B = 1 um^2/s, sigma = 5 nm,
kappa_a = 0.1 um^3/s, k_off = 10/s, dt = 10 us, binary32 state and displacements with
binary64 near-contact arguments.  One step = move, bin, pairs + p_enc, selection,
propagation/reaction, dissociation (the whole step of Sec. 3).

Prints one JSON line.  Kernel durations come from HIP events recorded on the
library's stream around every kernel of the timed steps.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(kernel, n_live, n_a, n_b, n_keys):
    """Bytes the method itself must move per launch of a stage (binary32 records): move 32 B per
    particle (read and write a position), binning 36 B per particle plus 8 B per bucket, the pair
    stage 32 B per A or B (new and old position)."""
    return {
        "move": 32 * n_live,
        "scan": 8 * n_keys,
        "scatter": 36 * n_live,
        "pairs": 32 * (n_a + n_b),
    }.get(kernel)


# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE on this workload (KiB per
# dispatch, each counter scaled by what it reads for a plain 256 MiB device copy); the table and the
# commands are in profiles/rad3d_step_traffic.md.  Valid only for the kernel sources they were taken
# on (hash below): after any change to them the field is reported as null.
MEASURED_TRAFFIC = {
    "src_hash": "1b95076bde67f42b",
    "scale_fetch": 1.9998, "scale_write": 1.0,
    "kib": {  # stage -> (FETCH_SIZE, WRITE_SIZE) summed over the stage's kernels
        "move": (9935.4, 31398.0),
        "scan": (11642.1, 17387.4),
        "scatter": (17008.8, 29448.9),
        "pairs": (9762.8, 299.2),
        "eval": (3255.2, 200.1),
        "select_a": (251.5, 60.5),
        "select_b": (269.3, 12.2),
        "events": (2.8, 0.9),  # k_close only: the 3D events run in the angle stage's kernel
    },
    # stage -> VALU wave-instructions per launch (SQ_INSTS_VALU summed over the stage's kernels)
    "valu": {
        "move": 6003796,
        "scan": 416342,
        "scatter": 723654,
        "pairs": 5250566,
        "eval": 437557,
        "select_a": 69692,
        "select_b": 214434,
        "events": 21,
    },
}


def _code_text(path):
    """A source file without its comments and with every run of white space made one blank:
    what the compiler reads, so that edits to comments leave the hashes below unchanged."""
    src = open(path, encoding="utf-8").read()
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":  # a literal, escapes included
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def _src_hash(files):
    h = hashlib.sha256()
    for f in files:
        h.update(_code_text(os.path.join(ROOT, "paper_1107_0270_amd", "csrc", f)).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def kernel_src_hash():
    return _src_hash(["common.hpp", "green.hpp", "kernels.hpp", "gfbd.hip"])


def measured_traffic(stage):
    t = MEASURED_TRAFFIC
    if stage not in t["kib"] or kernel_src_hash() != t["src_hash"]:
        return None
    f, w = t["kib"][stage]
    return int(f * 1024 * t["scale_fetch"] + w * 1024 * t["scale_write"])


# VALU issue peak: a wave64 VALU instruction occupies one of 256 CUs x 4 SIMDs for 4 cycles at 2.4 GHz
VALU_WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4


def valu_issue(stage, launch_ms):
    """The stage's measured VALU wave-instructions per launch (profiles/rad3d_step_valu.md), the
    time they take at the issue peak, and that time over the live launch duration."""
    t = MEASURED_TRAFFIC
    if stage not in t["valu"] or kernel_src_hash() != t["src_hash"]:
        return None
    n = t["valu"][stage]
    at_peak = n / VALU_WAVE_INSTR_PER_S * 1e3
    return {"wave_instructions_per_launch": n, "issue_ms_at_peak": round(at_peak, 5),
            "frac": round(at_peak / launch_ms, 4), "peak_wave_instr_per_s": VALU_WAVE_INSTR_PER_S}


# k_angle_wg on the --angle workloads (3D: 10^6 pairs, tau = 0.8; 2D: 2 x 10^5 pairs, tau = 0.04):
# fp64 operations and VALU wave-instructions per launch from rocprofv3
# (SQ_INSTS_VALU_{ADD,MUL,TRANS,FMA}_F64 x 64 lanes, an FMA counting two; SQ_INSTS_VALU),
# profiles/angle3_kernels.md and profiles/angle2_kernels.md.  Valid for the source they were taken on.
ANGLE_COUNTERS = {3: {
    "src_hash": "19e71876d53c5d1c",
    "pairs": 1000000,
    "f64_flop": 4.631595e+11,  # 64 x (ADD 459791425 + MUL 1741552687 + TRANS 164812436 + 2 x FMA 2435355467)
    "valu": 7445373893,
}, 2: {  # k_angle_wg<2> on --angle 200000 --dim 2 (membrane pairs, tau = 0.04)
    "src_hash": "e86c7c93a4030e22",
    "pairs": 200000,
    "f64_flop": 6.560815e+11,  # 64 x (ADD 602869869 + MUL 2437297157 + TRANS 198034386 + 2 x FMA 3506536180)
    "valu": 9468675080,
}}
FP64_VECTOR_PEAK = 78.6e12  # MI355X dense fp64 vector FLOP/s


def angle_src_hash(dim=3):
    return _src_hash(["angle3.hpp", "angle_wg.hpp"] + (["angle2.hpp"] if dim == 2 else []))


def angle_roofline(n, launch_ms, dim=3):
    """The angle kernel against the fp64 vector peak (its work is plain fp64 arithmetic: Bessel
    recurrences, quadrature sums, Legendre or sine sums), with the VALU issue fraction beside it."""
    t = ANGLE_COUNTERS[dim]
    if n != t["pairs"] or angle_src_hash(dim) != t["src_hash"]:
        return None
    achieved = t["f64_flop"] / (launch_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": round(achieved * 1e12 / FP64_VECTOR_PEAK, 4), "traffic": None,
            "flop_per_launch": t["f64_flop"], "flop_source": "rocprofv3 fp64 VALU counters (executed, not algorithmic)",
            "valu_issue_frac": round(t["valu"] / VALU_WAVE_INSTR_PER_S / (launch_ms * 1e-3), 4)}


# The step's angle stage on the default run of this workload (3D: k_events_angles, which runs each
# event and then the angle of its propagated pair; 2D: k_angles): fp64 operations and VALU
# wave-instructions per launch from rocprofv3 (SQ_INSTS_VALU_{ADD,MUL,TRANS,FMA}_F64 x 64 lanes, an
# FMA counting two; SQ_INSTS_VALU), and its HBM bytes (FETCH_SIZE, WRITE_SIZE scaled as above),
# profiles/rad3d_step_valu.md and profiles/rad3d_step_traffic.md.  Valid for the sources they were taken on (hash below).
ANGLE_STEP_COUNTERS = {
    "src_hash": "46853af3da5233a3",
    "f64_flop": 2.701000e+08,  # 64 x (ADD 425290 + MUL 845650 + TRANS 98717 + 2 x FMA 1425328)
    "valu": 4841123,
    "traffic": 1426467,
}
ANGLE_STEP_SOURCES = ["common.hpp", "green.hpp", "green2x.hpp", "kernels.hpp", "angle3.hpp", "angle2.hpp",
                      "angle_wg.hpp", "gfbd.hip"]


def angle_step_src_hash():
    return _src_hash(ANGLE_STEP_SOURCES)


def angle_step_roofline(launch_ms, profiled):
    """The angle stage against the fp64 vector peak: plain fp64 arithmetic (Bessel recurrences,
    quadrature sums, Legendre sums) on a few hundred pairs, a workgroup each (in 3D the same
    launch runs the step's events first, one wave each).  The operations are the ones the kernel
    executes (counters), not an algorithmic count."""
    t = ANGLE_STEP_COUNTERS
    valid = profiled and t["src_hash"] is not None and angle_step_src_hash() == t["src_hash"]
    out = {"kernel": "k_events_angles (the step's events, then the angles of its propagated pairs)", "bound": "alu", "achieved": None, "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
           "frac": None, "traffic": t["traffic"] if valid else None, "avg_launch_ms": round(launch_ms, 5),
           "flop_source": "rocprofv3 fp64 VALU counters of k_events_angles (events and angles; executed operations)",
           "valu_issue_frac": None}
    if valid:
        ach = t["f64_flop"] / (launch_ms * 1e-3) / 1e12
        out.update(achieved=round(ach, 3), frac=round(ach * 1e12 / FP64_VECTOR_PEAK, 4), flop_per_launch=t["f64_flop"],
                   valu_issue_frac=round(t["valu"] / VALU_WAVE_INSTR_PER_S / (launch_ms * 1e-3), 4))
    return out


def describe(cfg):
    bc = {0: "absorbing", 1: "reflecting", 2: "radiation"}[cfg["bc"]]
    rev = "reversible A+B<->C" if cfg["k_off"] > 0 else "irreversible A+B->C"
    k_units = "um^3/s" if cfg["dim"] == 3 else "um^2/s"
    return (f"{cfg['dim']}D {rev}, {bc} surface: {cfg['n_a']:g} A + {cfg['n_b']:g} B, periodic L={cfg['box']:g} um, "
            f"D={cfg['D'][0]:g} um^2/s, sigma={cfg['sigma'] * 1e3:g} nm, kappa={cfg['kappa_a']:g} {k_units}, "
            f"k_off={cfg['k_off']:g}/s, dt={cfg['dt'] * 1e6:g} us")


def pair_probs(args, I, S):
    print(json.dumps(pair_probs_record(args.pair_probs, args.steps, args.dim, I, S)), flush=True)


def pair_probs_record(n, repeats, d, I, S):
    """p_enc and p_reac of N pairs drawn from the workload's pair distribution (uniform positions:
    R uniform in the ball of radius r_cut/a; R0 = |R + sqrt(2 tau) z| >= 1, z standard normal),
    evaluated by sim_eval_pairs with the step's device functions on device-resident arrays."""
    cfg = I.workload("cfg_rad3d" if d == 3 else "cfg_mem2d_small_tau")
    sp = np.array([0, 1], np.int32)
    pos = np.array([[0.25] * d, [0.75] * d])
    h = S.Sim(dim=d, box=cfg["box"], dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"], bc=cfg["bc"], kappa=cfg["kappa_a"],
              k_off=0.0, precision=cfg["precision"], seed=0, species=sp, pos=pos, eps_cut=1e-6)
    der = h.derived()
    tau, rmax = der["tau"], der["rcut"] / der["a"]
    rng = np.random.default_rng(0)
    v = rng.standard_normal((n, d))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    v *= (rmax * rng.random(n) ** (1.0 / d))[:, None]
    R = np.linalg.norm(v, axis=1)
    v += np.sqrt(2.0 * tau) * rng.standard_normal((n, d))
    R0 = np.maximum(np.linalg.norm(v, axis=1), 1.0)
    del v
    bufs = [S.DeviceBuffer(8 * n) for _ in range(4)]
    bufs[0].upload(R)
    bufs[1].upload(R0)
    out = {}
    for name, want_preac in (("penc", False), ("penc_preac", True)):
        args4 = (n, bufs[0].ptr, bufs[1].ptr, bufs[2].ptr, bufs[3].ptr if want_preac else None)
        h.eval_pairs_device(*args4)  # warm-up
        t0 = time.perf_counter()
        for _ in range(repeats):
            h.eval_pairs_device(*args4)
        out[name] = n * repeats / (time.perf_counter() - t0)
        log(f"[pair-probs] {name}: {out[name]:.3e} pair evals/s")
    for b in bufs:
        b.free()
    h.close()
    return {
        "metric": "pair-probability evals/s (kernel only)", "value": round(out["penc"], 1), "unit": "pair evals/s",
        "penc_and_preac_per_s": round(out["penc_preac"], 1), "n_gpus": 1, "pairs": n, "repeats": repeats,
        "dtype": {0: "f64", 1: "f32", 2: "f32+f64-args", 3: "f32+f64-args"}[cfg["precision"]], "data": "synthetic",
        "config": {"workload": f"{d}D pair distribution of the benchmark workload at the 1e-6 cut-off: R uniform in "
                               f"the ball of radius r_cut/a = {rmax:.3f}, R0 = |R + sqrt(2 tau) z|, tau = {tau:.4g}",
                   "kernel": "k_eval_probs (the step's p_enc / p_reac device functions)"}}


def first_passage(args, I, S):
    """First contact of N candidate pairs of the benchmark workload (3D, or the 2D membrane
    workload at tau = 0.04 with --dim 2) located by bisection
    (sim_eval_first_passage, the paper's Appendix) to dt / 2^levels, on device-resident arrays.
    Candidates: a pre-step separation uniform in the shell 1 < R0 < r_cut/a, a free step of
    sqrt(2 tau) z, kept with the encounter probability that the step's own device function gives
    (sim_eval_pairs), as the step keeps its candidates."""
    dim = args.dim
    cfg = I.workload("cfg_rad3d" if dim == 3 else "cfg_mem2d_small_tau")
    sp = np.array([0, 1], np.int32)
    pos = np.array([[0.25] * dim, [0.75] * dim])
    h = S.Sim(dim=dim, box=cfg["box"], dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"], bc=cfg["bc"], kappa=cfg["kappa_a"],
              k_off=0.0, precision=S.PREC_FP64, seed=0, species=sp, pos=pos)
    der = h.derived()
    tau, rmax, n, levels = der["tau"], der["rcut"] / der["a"], args.first_passage, args.fp_levels
    rng = np.random.default_rng(0)
    xi_all, xf_all, have = [], [], 0
    while have < n:
        m = 4 * n
        d = rng.standard_normal((m, dim))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        xi = d * ((1.0 + (rmax ** dim - 1.0) * rng.random(m)) ** (1.0 / dim))[:, None]
        xf = xi + np.sqrt(2.0 * tau) * rng.standard_normal((m, dim))
        if dim == 2:  # the boundary takes three components per pair
            xi, xf = np.pad(xi, ((0, 0), (0, 1))), np.pad(xf, ((0, 0), (0, 1)))
        R, R0 = np.ascontiguousarray(np.linalg.norm(xf, axis=1)), np.ascontiguousarray(np.linalg.norm(xi, axis=1))
        bR, bR0, bp = S.DeviceBuffer(8 * m), S.DeviceBuffer(8 * m), S.DeviceBuffer(8 * m)
        bR.upload(R)
        bR0.upload(R0)
        h.eval_pairs_device(m, bR.ptr, bR0.ptr, bp.ptr, None)
        p = bp.download(np.empty(m, np.float64))
        for b in (bR, bR0, bp):
            b.free()
        keep = rng.random(m) < p
        xi_all.append(xi[keep])
        xf_all.append(xf[keep])
        have += int(keep.sum())
    xi = np.ascontiguousarray(np.concatenate(xi_all)[:n])
    xf = np.ascontiguousarray(np.concatenate(xf_all)[:n])
    bi, bf, blo, ba = S.DeviceBuffer(24 * n), S.DeviceBuffer(24 * n), S.DeviceBuffer(8 * n), S.DeviceBuffer(4 * n)
    bi.upload(xi)
    bf.upload(xf)
    call = (n, bi.ptr, bf.ptr, levels, 1, blo.ptr, ba.ptr)
    h.eval_first_passage_device(*call)  # warm-up
    t0 = time.perf_counter()
    for _ in range(args.steps):
        h.eval_first_passage_device(*call)
    el = time.perf_counter() - t0
    att = ba.download(np.empty(n, np.uint32))
    lo = blo.download(np.empty(n, np.uint64))
    for b in (bi, bf, blo, ba):
        b.free()
    h.close()
    rate = n * args.steps / el
    cpu = None
    if args.cpu_steps > 0:
        import oracle as O

        m = min(n, 20000)
        key = (0, 0)  # seed 0, replica 0
        tc = time.perf_counter()
        for k in range(m):
            O.first_passage(dim, xi[k][:dim], xf[k][:dim], tau, levels, k, 1, key)
        tc = time.perf_counter() - tc
        cpu = {"value": round(m / tc, 1), "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {m} of the same candidates, one call of the single-threaded FP64 C oracle each "
                         f"({tc:.1f} s)"}
        log(f"[first-passage] cpu baseline {cpu}")
    frac_first = float(np.mean(lo < (1 << (levels - 1))))
    exhausted = (att & 0x80000000) != 0
    props = float(np.mean(att & 0x7FFFFFFF))
    log(f"[first-passage] {n} pairs x {levels} levels: {rate:.3e} pairs/s, {props:.2f} proposals per pair, "
        f"{exhausted.mean():.2e} of the pairs exhausted a level, first contact in the first half of the step "
        f"for {frac_first:.3f}")
    print(json.dumps({
        "metric": "first-passage refinements/s (kernel only)", "value": round(rate, 1), "unit": "pairs/s",
        "levels_per_s": round(rate * levels, 1), "proposals_per_pair": round(props, 3),
        "exhausted_fraction": float(exhausted.mean()), "cpu_baseline": cpu,
        "n_gpus": 1, "pairs": n, "levels": levels, "repeats": args.steps, "ms_per_call": round(el * 1e3 / args.steps, 4),
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{dim}D candidates of the benchmark workload: R0 uniform in the shell 1 < R0 < r_cut/a = "
                               f"{rmax:.3f}, R = R0 + sqrt(2 tau) z, kept with p_enc(R, R0), tau = {tau:.4g}; first "
                               f"contact located to dt / 2^{levels}",
                   "kernel": "k_first_passage (bisection of the Appendix, 16 lanes per pair)"}}), flush=True)


def angle(args, I, S):
    """Angles of N propagated pairs of the benchmark workload (sim_eval_angle: cos Theta from
    J (G_ref - G_abs) given the radii, Sec. 3, Details, eq. genericGF3D), on device-resident
    arrays.  Pairs: a pre-step separation uniform in the shell 1 < R0 < r_cut/a, the new radius
    drawn from the radial propagator by the step's own sampler (sim_eval_propagator), a uniform u."""
    dim = args.dim
    cfg = I.workload("cfg_rad3d" if dim == 3 else "cfg_mem2d_small_tau")
    sp = np.array([0, 1], np.int32)
    pos = np.array([[0.25] * dim, [0.75] * dim])
    h = S.Sim(dim=dim, box=cfg["box"], dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"], bc=cfg["bc"], kappa=cfg["kappa_a"],
              k_off=0.0, precision=S.PREC_FP64, seed=0, species=sp, pos=pos)
    der = h.derived()
    tau, rmax, n = der["tau"], der["rcut"] / der["a"], args.angle
    rng = np.random.default_rng(0)
    R0 = np.ascontiguousarray((1.0 + (rmax ** dim - 1.0) * rng.random(n)) ** (1.0 / dim))
    u = rng.random(n)
    bR, bR0, bu, bc = (S.DeviceBuffer(8 * n) for _ in range(4))
    bR0.upload(R0)
    bu.upload(u)
    h.eval_propagator_device(n, bR0.ptr, 1, 0, bR.ptr, None)
    call = (n, bR.ptr, bR0.ptr, bu.ptr, bc.ptr)
    h.eval_angle_device(*call)  # warm-up
    t0 = time.perf_counter()
    for _ in range(args.steps):
        h.eval_angle_device(*call)
    el = time.perf_counter() - t0  # each call returns when its launch is done
    R = bR.download(np.empty(n))
    c = bc.download(np.empty(n))
    for b in (bR, bR0, bu, bc):
        b.free()
    h.close()
    rate = n * args.steps / el
    cpu = None
    if args.cpu_steps > 0:
        import oracle as O

        m = min(n, 20000)
        tc = time.perf_counter()
        k = 0
        while k < m and time.perf_counter() - tc < 20.0:
            (O.sample_angle3 if dim == 3 else O.sample_angle2)(R[k], R0[k], tau, u[k])
            k += 1
        tc = time.perf_counter() - tc
        cpu = {"value": round(k / tc, 1), "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {k} of the same pairs, one call of the single-threaded FP64 C oracle each "
                         f"({tc:.1f} s)"}
        log(f"[angle] cpu baseline {cpu}")
    what = "cos_theta" if dim == 3 else "abs_theta"
    log(f"[angle] {n} pairs: {rate:.3e} pairs/s, mean {what} {c.mean():.4f}, mean R'' {R.mean():.4f}")
    print(json.dumps({
        "metric": "propagated-pair angles/s (kernel only)", "value": round(rate, 1), "unit": "pairs/s",
        f"mean_{what}": round(float(c.mean()), 6),
        "roofline": angle_roofline(n, el * 1e3 / args.steps, dim),
        "cpu_baseline": cpu,
        "n_gpus": 1, "pairs": n, "repeats": args.steps, "ms_per_call": round(el * 1e3 / args.steps, 4),
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{dim}D propagated pairs of the {'benchmark' if dim == 3 else 'membrane'} workload: "
                               f"R0 uniform in the {'shell' if dim == 3 else 'ring'} 1 < R0 < r_cut/a = {rmax:.3f}, "
                               f"R'' from the radial propagator, tau = {tau:.4g}",
                   "kernel": "k_angle_wg<3> (Legendre series of G_ref - G_abs, one workgroup per pair)" if dim == 3 else
                             "k_angle_wg<2> (cos(n theta) series of G_ref - G_abs, one workgroup per pair)"}}), flush=True)


def batched(args, I, S):
    """R independent 3D replicas stepped together (sim_batch_create, one graph replay per step)
    against the plain path: a sample of the same replicas stepped one handle at a time."""
    shared = dict(dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, bc=S.BC_RADIATION, k_off=10.0, seed=0, eps_cut=args.eps_cut,
                  precision=S.PREC_FP32D_FP64NC)
    t0 = time.time()
    reps = I.ensemble(args.batch)
    n_tot = sum(len(r["species"]) for r in reps)
    log(f"[batch] {len(reps)} replicas, {n_tot} particles, generated in {time.time() - t0:.1f}s")
    tuned = None
    if args.autotune:
        # replicas share the density, so a sub-batch picks the shared cell edge (batches use the
        # direct pair search)
        from paper_1107_0270_amd import autotune as AT
        rng0 = np.random.default_rng(2)
        sub = [reps[i] for i in rng0.choice(len(reps), size=min(256, len(reps)), replace=False)]
        probe = S.Sim.batch(sub[:1], **shared)
        d0 = probe.derived()
        probe.close()
        t0 = time.time()
        best, table = AT.tune(lambda c, p, **launch: S.Sim.batch(sub, cell=c, **launch, **shared), box=sub[0]["box"],
                              dim=3, rcut=d0["rcut"], cell0=d0["cell"], searches=(S.PAIRS_DIRECT,), log=log)
        shared.update(cell=best["cell"], pair_blocks=best["pair_blocks"], event_blocks=best["event_blocks"])
        tuned = {"choice": best, "tuned_on": f"{len(sub)} replicas of the ensemble", "candidates": len(table),
                 "seconds": round(time.time() - t0, 1),
                 "table": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()} for r in table]}
        log(f"[batch] autotuned in {tuned['seconds']} s: {best}")
    t0 = time.time()
    b = S.Sim.batch(reps, **shared)
    log(f"[batch] created in {time.time() - t0:.1f}s")
    b.step(args.warmup)
    c0 = b.counts()
    t0 = time.perf_counter()
    b.step(args.steps)
    el = time.perf_counter() - t0
    c1 = b.counts()
    b.close()
    n_live = 0.5 * sum(c0[k] + c1[k] for k in ("A", "B", "C"))
    rate = n_live * args.steps / el
    log(f"[batch] {args.steps} steps in {el * 1e3:.1f} ms: {rate:.3e} particle-steps/s")
    # plain path: the same replicas, one handle each, stepped one after another
    rng = np.random.default_rng(1)
    pick = rng.choice(len(reps), size=min(args.single_sample, len(reps)), replace=False)
    t_single, ps_single = 0.0, 0.0
    for r in pick:
        rd = reps[r]
        sim = S.Sim(dim=3, box=rd["box"], species=rd["species"], pos=rd["pos"], kappa=rd["kappa"],
                    replica=rd["replica"], **shared)
        sim.step(args.warmup)
        t0 = time.perf_counter()
        sim.step(args.steps)
        t_single += time.perf_counter() - t0
        ps_single += len(rd["species"]) * args.steps
        sim.close()
    rate1 = ps_single / t_single
    log(f"[batch] single-replica path on {len(pick)} replicas: {rate1:.3e} particle-steps/s")
    print(json.dumps({
        "metric": "particle-steps/s (batched ensemble)", "value": round(rate, 1), "unit": "particle-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(el * 1e3 / args.steps, 4),
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "single_replica_path": {"value": round(rate1, 1), "unit": "particle-steps/s",
                                "sample": f"{len(pick)} replicas of the ensemble, one handle each, stepped one after "
                                          f"another ({args.steps} steps each after {args.warmup} warm-up)"},
        "speedup_vs_single_replica_path": round(rate / rate1, 2),
        "autotune": tuned,
        "config": {"workload": f"{len(reps)} independent 3D replicas, A+B<->C radiation surface, N log-uniform in "
                               f"[1e3, 1e5] (total {n_tot}), kappa uniform in [0.01, 1] um^3/s, L = (N/1000)^(1/3) um, "
                               "D=1 um^2/s, sigma=5 nm, k_off=10/s, dt=10 us",
                   "precision": "binary32 state and p_enc, binary64 near-contact arguments and propagation",
                   "step_launch": "one hipGraph replay per step for all replicas"}}), flush=True)


ENSEMBLE_SHARED = dict(dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, k_off=10.0, seed=0, eps_cut=1e-6)


def ensemble_record(reps, S, steps=50, warmup=5, sample=16):
    """The batched ensemble (one graph replay per step for all replicas) and the plain path on a
    sample of the same replicas, one handle each, for the default benchmark line."""
    shared = dict(ENSEMBLE_SHARED, bc=S.BC_RADIATION, precision=S.PREC_FP32D_FP64NC)
    n_tot = sum(len(r["species"]) for r in reps)
    t0 = time.time()
    b = S.Sim.batch(reps, **shared)
    t_create = time.time() - t0
    b.step(warmup)
    c0 = b.counts()
    t0 = time.perf_counter()
    b.step(steps)
    el = time.perf_counter() - t0
    c1 = b.counts()
    b.close()
    rate = 0.5 * sum(c0[k] + c1[k] for k in ("A", "B", "C")) * steps / el
    rng = np.random.default_rng(1)
    t1, ps1 = 0.0, 0.0
    for r in rng.choice(len(reps), size=min(sample, len(reps)), replace=False):
        rd = reps[r]
        sim = S.Sim(dim=3, box=rd["box"], species=rd["species"], pos=rd["pos"], kappa=rd["kappa"], replica=rd["replica"],
                    **shared)
        sim.step(warmup)
        t0 = time.perf_counter()
        sim.step(steps)
        t1 += time.perf_counter() - t0
        ps1 += len(rd["species"]) * steps
        sim.close()
    log(f"[bench] ensemble: {rate:.3e} particle-steps/s; plain path {ps1 / t1:.3e}")
    return {"value": round(rate, 1), "unit": "particle-steps/s", "ms_per_step": round(el * 1e3 / steps, 4),
            "steps": steps, "warmup": warmup, "handle_creation_s": round(t_create, 2),
            "plain_path": {"value": round(ps1 / t1, 1), "unit": "particle-steps/s",
                           "sample": f"{min(sample, len(reps))} replicas of the ensemble, one handle each, "
                                     f"{steps} steps each after {warmup} warm-up"},
            "speedup_vs_plain_path": round(rate * t1 / ps1, 2),
            "workload": f"{len(reps)} independent 3D replicas, A+B<->C radiation surface, N log-uniform in [1e3, 1e5] "
                        f"(total {n_tot}), kappa uniform in [0.01, 1] um^3/s, L = (N/1000)^(1/3) um, D=1 um^2/s, "
                        "sigma=5 nm, k_off=10/s, dt=10 us, binary32 state and displacements with binary64 "
                        "near-contact arguments, pair cut-off 1e-6"}


SERVE_HBM_BUDGET = 32 << 30  # the served stream's ledger: device bytes of running requests, both pools


def served_record(trace, S, pool_slots=1 << 26, tick=200, sample=8):
    """The served stream on a given (shortened) trace: p50/p99 latency and aggregate
    particle-steps/s, against the plain path on a sample of its requests."""
    from paper_1107_0270_amd import serve as V
    work = sum(r.n * r.steps for r in trace)
    rng = np.random.default_rng(1)
    t1, ps1 = 0.0, 0
    for i in rng.choice(len(trace), size=min(sample, len(trace)), replace=False):
        r = trace[i]
        p = dict(V.GROUP_PARAMS[r.dim])
        dim = p.pop("dim")
        sim = S.Sim(dim=dim, box=r.box, species=r.species, pos=r.pos, replica=r.id, **p)
        k = min(r.steps, 200)
        t0 = time.perf_counter()
        sim.step(k)
        t1 += time.perf_counter() - t0
        ps1 += r.n * k
        sim.close()
    srv = V.Server(slot_cap={3: pool_slots, 2: pool_slots}, tick=tick, keep_results=False, read_results=True,
                   progress=None, hbm_budget=SERVE_HBM_BUDGET)
    srv.run(trace)
    summ = srv.summary(trace)
    log(f"[bench] served: {summ}")
    return {"value": round(summ["particle_steps_per_s"], 1), "unit": "particle-steps/s",
            "p50_latency_s": round(summ["p50_latency_s"], 4), "p99_latency_s": round(summ["p99_latency_s"], 4),
            "mean_queue_s": round(summ["mean_queue_s"], 4), "wall_s": round(summ["wall_s"], 3),
            "offered_particle_steps_per_s": round(work / trace[-1].arrival, 1),
            "plain_path": {"value": round(ps1 / t1, 1), "unit": "particle-steps/s",
                           "sample": f"{min(sample, len(trace))} requests of the trace, one handle each, at most 200 "
                                     "steps each"},
            "speedup_vs_plain_path": round(summ["particle_steps_per_s"] * t1 / ps1, 2),
            "workload": f"shortened served stream: the first {len(trace)} requests of the Poisson trace at 200 req/s "
                        "(seed 0); 3D or 2D with p = 1/2; N log-uniform in [1e3, 1e6]; steps log-uniform in "
                        "[100, 1e4]; overlapping A-B pairs redrawn; 3D: the headline parameters; 2D: D=0.1 um^2/s, "
                        "kappa=0.05 um^2/s, k_off=10/s, dt=5 us; pair cut-off 1e-6",
            "admission": f"one pool per dimension of {pool_slots} slots; an HBM ledger of {SERVE_HBM_BUDGET >> 30} GiB "
                         f"for both ({V.BYTES_PER_SLOT} B per particle); arrival order with at most {srv.max_bypass} "
                         f"later requests admitted ahead of one that does not fit; each pool steps to its next "
                         f"completion, at most {tick} steps per call",
            "bypasses": summ["bypasses"], "ledger_peak_bytes": summ["ledger_peak_bytes"]}


def _oracle_worker(payload):
    """One oracle on its own core (a spawned process that never touches the GPU)."""
    cfg, sp, pos, box, steps, eps = payload
    sys.path.insert(0, ROOT)
    import oracle as O
    orc = O.OracleSim(dim=cfg["dim"], bc=cfg["bc"], box=[box] * cfg["dim"], dt=cfg["dt"], D=cfg["D"],
                      sigma=cfg["sigma"], kappa_a=cfg["kappa_a"], k_off=cfg["k_off"], store_f32=cfg["precision"] != 0,
                      eps_cut=eps, species=sp, pos=pos)
    t0 = time.perf_counter()
    orc.step(steps)
    return time.perf_counter() - t0


def cpu_baselines(cfg, sp, pos, box, steps, eps):
    """The FP64 oracle as it stands on the same workload and initial state: one process on one
    core, and one process per available core (up to 16, the box's share) each stepping its own copy
    at once.  Runs before the benchmark touches the GPU (the workers are spawned processes)."""
    import multiprocessing as mp
    payload = (cfg, sp, pos, box, steps, eps)
    t1 = _oracle_worker(payload)
    single = {"value": round(len(sp) * steps / t1, 1), "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
              "sample": f"{steps} steps of the same {len(sp)}-particle workload from the same initial state, "
                        f"single-threaded FP64 C oracle ({t1:.1f} s)"}
    log(f"[bench] cpu baseline, one core: {single}")
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(16, cores))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        times = pool.map(_oracle_worker, [payload] * cores)
    wall = time.perf_counter() - t0
    rate = cores * len(sp) * steps / max(times)
    log(f"[bench] cpu baseline, {cores} cores: {rate:.3e} particle-steps/s (slowest worker {max(times):.1f} s, "
        f"wall {wall:.1f} s)")
    return {"value": round(rate, 1), "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} copies of the same {len(sp)}-particle workload, {steps} steps each from the same "
                      f"initial state, one single-threaded FP64 C oracle per core at once (slowest {max(times):.1f} s)",
            "single_core": single}


def served(args, S):
    """The served stream: Poisson arrivals of 2D/3D reversible simulations (N and steps
    log-uniform), continuous batching in one pool per dimension; p50/p99 latency and aggregate
    particle-steps/s, against the plain path (requests run alone, one after another)."""
    from paper_1107_0270_amd import serve as V
    trace = V.make_trace(args.serve_requests, args.serve, seed=0)
    t0 = time.time()
    for r in trace:
        V.initial_state(r)
    n_tot = sum(r.n for r in trace)
    work = sum(r.n * r.steps for r in trace)
    log(f"[serve] {len(trace)} requests at {args.serve}/s: {n_tot} particles, {work:.3e} particle-steps, "
        f"states in {time.time() - t0:.1f}s")
    # plain path first (also warms the library): a sample of the requests, one handle each
    rng = np.random.default_rng(1)
    pick = rng.choice(len(trace), size=min(args.single_sample, len(trace)), replace=False)
    t_single, ps_single = 0.0, 0
    for i in pick:
        r = trace[i]
        p = dict(V.GROUP_PARAMS[r.dim])
        dim = p.pop("dim")
        sim = S.Sim(dim=dim, box=r.box, species=r.species, pos=r.pos, replica=r.id, **p)
        k = min(r.steps, 200)
        t1 = time.perf_counter()
        sim.step(k)
        t_single += time.perf_counter() - t1
        ps_single += r.n * k
        sim.close()
    rate1 = ps_single / t_single
    log(f"[serve] plain path on {len(pick)} requests: {rate1:.3e} particle-steps/s")
    srv = V.Server(slot_cap={3: args.pool_slots, 2: args.pool_slots}, tick=args.tick, keep_results=False,
                   read_results=True, progress=log, hbm_budget=SERVE_HBM_BUDGET)
    srv.run(trace)
    summ = srv.summary(trace)
    log(f"[serve] {summ}")
    lat = np.array([r.finished - r.arrival for r in trace])
    print(json.dumps({
        "metric": "p50/p99 request latency; aggregate particle-steps/s (served stream)",
        "value": round(summ["particle_steps_per_s"], 1), "unit": "particle-steps/s",
        "p50_latency_s": round(summ["p50_latency_s"], 4), "p99_latency_s": round(summ["p99_latency_s"], 4),
        "mean_queue_s": round(summ["mean_queue_s"], 4),
        "mean_service_s": round(float(np.mean([r.finished - r.admitted for r in trace])), 4),
        "wall_s": round(summ["wall_s"], 3), "last_arrival_s": round(trace[-1].arrival, 3),
        "offered_particle_steps_per_s": round(work / trace[-1].arrival, 1),
        "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "plain_path": {"value": round(rate1, 1), "unit": "particle-steps/s",
                       "sample": f"{len(pick)} requests of the trace, one handle each, run one after another "
                                 "(at most 200 steps each)"},
        "speedup_vs_plain_path": round(summ["particle_steps_per_s"] / rate1, 2),
        "latency_quantiles_s": {q: round(float(np.percentile(lat, q)), 4) for q in (10, 25, 50, 75, 90, 99)},
        "server": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()},
        "config": {"workload": f"{len(trace)} requests, Poisson arrivals at {args.serve}/s (seed 0); 3D or 2D with "
                               "p = 1/2; N log-uniform in [1e3, 1e6]; steps log-uniform in [100, 1e4]; 3D: D=1 um^2/s, "
                               "sigma=5 nm, kappa=0.1 um^3/s, k_off=10/s, dt=10 us, 1000 particles/um^3; 2D: D=0.1 "
                               "um^2/s, kappa=0.05 um^2/s, k_off=10/s, dt=5 us, 2500 particles/um^2",
                   "admission": f"first come first served into one pool per dimension of {args.pool_slots} slots "
                                "(the device-memory ledger); each request occupies its own slot and cell ranges "
                                "until it finishes",
                   "tick": f"each pool steps to its next completion, at most {args.tick} steps per call",
                   "precision": "binary32 state and p_enc, binary64 near-contact arguments and propagation"}}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=30,
                    help="oracle steps timed for the CPU baselines, on one core and on each core (0 = skip)")
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="leave the ensemble, the shortened served stream and the pair-probability rate out of the line")
    ap.add_argument("--serve-requests-short", type=int, default=100,
                    help="requests of the shortened served stream in the default line")
    ap.add_argument("--no-timing", action="store_true", help="time without per-kernel events")
    ap.add_argument("--pair-search", choices=["auto", "bricks", "direct"], default="auto",
                    help="pair-search kernel (auto = the library's choice)")
    ap.add_argument("--cell", type=float, default=0.0, help="cell edge in um (0 = the library's choice)")
    ap.add_argument("--workload", default="cfg_rad3d",
                    choices=["cfg_rad3d", "cfg_rad3d_dense", "cfg_mem2d", "cfg_mem2d_small_tau", "cfg_abs3d"],
                    help="synthetic workload (default: the 3D radiation workload the metric is quoted on)")
    ap.add_argument("--first-passage", type=int, default=0, metavar="N",
                    help="time the first-passage bisection on N candidate pairs instead of the step")
    ap.add_argument("--fp-levels", type=int, default=20, help="bisection levels for --first-passage")
    ap.add_argument("--angle", type=int, default=0, metavar="N",
                    help="time the 3D angular propagator on N propagated pairs instead of the step")
    ap.add_argument("--pair-probs", type=int, default=0, metavar="N",
                    help="only run the pair-probability micro-benchmark on N synthetic pairs and exit")
    ap.add_argument("--dim", type=int, default=3, help="workload dimension for --pair-probs, --first-passage and "
                    "--angle (2: the membrane workload at dt = 5 us)")
    ap.add_argument("--batch", type=int, default=0, metavar="R",
                    help="only run the batched-ensemble benchmark on R replicas (4096: the full ensemble) and exit")
    ap.add_argument("--single-sample", type=int, default=32,
                    help="replicas timed one handle at a time for the single-replica comparison (--batch)")
    ap.add_argument("--serve", type=float, default=0.0, metavar="RATE",
                    help="only run the served stream at RATE requests/s (200: the stated stream) and exit")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests in the served trace (--serve)")
    ap.add_argument("--pool-slots", type=int, default=1 << 26, help="slots of each pool (--serve)")
    ap.add_argument("--tick", type=int, default=200, help="most steps per pool call (--serve)")
    ap.add_argument("--precision", choices=["workload", "fp64", "fp32", "fp32nc", "fp32d"], default="workload",
                    help="precision mode (default: the workload's; fp32 = plain binary32, fp32nc = binary32 with "
                         "binary64 near-contact arguments and displacements, fp32d = fp32nc with binary32 "
                         "displacements)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain binary32 and binary32-displacement comparison runs")
    ap.add_argument("--green2d", choices=["auto", "expansion", "exact"], default="auto",
                    help="2D radial functions: small-time expansions, or exact (tables by quadrature); auto takes "
                         "the expansion where it holds the probabilities to 1e-6 (tau <= 0.05 at order 12) and "
                         "the exact functions beyond (the membrane workload as written, tau = 0.8)")
    ap.add_argument("--unvalidated-tau", action="store_true",
                    help="for timing comparisons only: accept the 2D small-time expansion beyond the tau where it "
                         "holds 1e-6 (the probabilities are then wrong; the line says so in config)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the cell edge and pair-search kernel by timing candidates on the workload first")
    ap.add_argument("--eps-cut", type=float, default=1e-6,
                    help="pair cut-off: pairs whose reaction probability within a step is below this are left out "
                         "(default 1e-6, the metric's probability accuracy; the paper's own cut-off is 1e-3)")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="particle count and box volume times this factor (same density; the metric is quoted at 1)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        x = torch.ones(args.copy_probe << 18, device="cuda")  # float32: MIB MiB
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": x.numel() * 4, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not supported", "n_gpus": args.gpus}))
        sys.exit(2)

    from paper_1107_0270_amd import inputs as I

    if args.pair_probs or args.first_passage or args.angle or args.batch or args.serve:
        from paper_1107_0270_amd import sim as S
        if args.pair_probs:
            pair_probs(args, I, S)
        elif args.first_passage:
            first_passage(args, I, S)
        elif args.angle:
            angle(args, I, S)
        elif args.batch:
            batched(args, I, S)
        else:
            served(args, S)
        return

    cfg = I.workload(args.workload)
    if args.precision != "workload":
        cfg["precision"] = {"fp64": I.PREC_FP64, "fp32": I.PREC_FP32, "fp32nc": I.PREC_FP32_FP64NC,
                            "fp32d": I.PREC_FP32D_FP64NC}[args.precision]
    dim = cfg["dim"]
    t0 = time.time()
    sp, pos, box, red = I.state_for(cfg, seed=0, scale=args.scale)
    if args.scale != 1.0:  # the same density in a box scaled with the particle count
        cfg = dict(cfg, n_a=int(np.sum(sp == I.SP_A)), n_b=int(np.sum(sp == I.SP_B)), box=box)
    log(f"[bench] state: {len(sp)} particles, {red} redrawn overlaps, {time.time() - t0:.1f}s")
    # the oracle on the host's cores first: its worker processes start before anything here
    # touches the GPU
    cpu = cpu_baselines(cfg, sp, pos, box, args.cpu_steps, args.eps_cut) if args.cpu_steps > 0 else None
    # the default line also reports the ensemble and a shortened served stream: their inputs are
    # generated on the host while the headline runs on the device
    extras = {}
    gen = None
    if args.extras:
        import threading

        def _generate():
            from paper_1107_0270_amd import serve as V
            t = time.time()
            extras["reps"] = I.ensemble(4096)
            trace = V.make_trace(args.serve_requests_short, 200.0, seed=0)
            for r in trace:
                V.initial_state(r, redraw=True)
            extras["trace"] = trace
            log(f"[bench] ensemble and trace inputs in {time.time() - t:.1f}s")

        gen = threading.Thread(target=_generate)
        gen.start()
    from paper_1107_0270_amd import sim as S
    search = {"auto": S.PAIRS_AUTO, "bricks": S.PAIRS_BRICKS, "direct": S.PAIRS_DIRECT}[args.pair_search]

    tau = (cfg["D"][0] + cfg["D"][1]) * cfg["dt"] / cfg["sigma"] ** 2
    if args.green2d == "auto":
        args.green2d = "exact" if dim == 2 and tau > 0.05 * (1 + 1e-9) else "expansion"
    g2 = S.G2_EXACT if args.green2d == "exact" else S.G2_EXPANSION
    g2_flags = S.F_UNVALIDATED_TAU if args.unvalidated_tau else 0

    launch = {}  # pair-stage and event workgroups (the library's defaults unless tuned)

    def make_with(timing, cell, pair_search, **shape):
        return S.Sim(dim=dim, box=box, dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"], bc=cfg["bc"], kappa=cfg["kappa_a"],
                     k_off=cfg["k_off"], precision=cfg["precision"], seed=0, species=sp, pos=pos, timing=timing, cell=cell,
                     pair_search=pair_search, green2d=g2, eps_cut=args.eps_cut, flags=g2_flags, **shape)

    tuned = None
    if args.autotune:
        from paper_1107_0270_amd import autotune as AT
        probe = make_with(False, 0.0, S.PAIRS_AUTO)
        d0 = probe.derived()
        probe.close()
        t0 = time.time()
        best, table = AT.tune(lambda c, p, **shape: make_with(False, c, p, **shape), box=box, dim=dim, rcut=d0["rcut"],
                              cell0=d0["cell"], log=log)
        args.cell, search = best["cell"], best["pair_search"]
        launch.update(pair_blocks=best["pair_blocks"], event_blocks=best["event_blocks"])
        tuned = {"choice": best, "candidates": len(table), "seconds": round(time.time() - t0, 1),
                 "table": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()} for r in table]}
        log(f"[bench] autotuned in {tuned['seconds']} s: {best}")

    def make(timing, precision=None):
        if precision is None:
            return make_with(timing, args.cell, search, **launch)
        return S.Sim(dim=dim, box=box, dt=cfg["dt"], D=cfg["D"], sigma=cfg["sigma"], bc=cfg["bc"], kappa=cfg["kappa_a"],
                     k_off=cfg["k_off"], precision=precision, seed=0, species=sp, pos=pos, timing=timing, cell=args.cell,
                     pair_search=search, green2d=g2, eps_cut=args.eps_cut, flags=g2_flags, **launch)

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
    t_create = time.perf_counter()
    sim = make(False)
    t_create = time.perf_counter() - t_create
    der, grid = sim.derived(), sim.grid()
    log(f"[bench] derived {der} grid {grid}")
    el, n_live, pairs, c0, c1, _ = timed(sim)
    sim.close()
    ps = n_live * args.steps / el
    log(f"[bench] graph: {args.steps} steps in {el * 1e3:.1f} ms; {ps:.3e} particle-steps/s; {pairs / el:.3e} pair evals/s")
    # the same workload in the plain binary32 mode (binary32 displacements and p_enc)
    plain = fp32d = None
    if cfg["precision"] in (S.PREC_FP32_FP64NC, S.PREC_FP32D_FP64NC) and not args.no_plain:
        sim = make(False, S.PREC_FP32)
        el32, n32, pairs32, _, _, _ = timed(sim)
        sim.close()
        plain = {"value": round(n32 * args.steps / el32, 1), "unit": "particle-steps/s",
                 "ms_per_step": round(el32 * 1e3 / args.steps, 5), "pair_evals_per_s": round(pairs32 / el32, 1),
                 "precision": "binary32 state, displacements, pair test and p_enc; binary64 propagation"}
        log(f"[bench] plain binary32: {plain}")
        # the other near-contact mode: binary64 displacements (bit-identical trajectories to the
        # oracle's) when the headline takes binary32 ones, and the reverse
        other = S.PREC_FP32_FP64NC if cfg["precision"] == S.PREC_FP32D_FP64NC else S.PREC_FP32D_FP64NC
        sim = make(False, other)
        elo, no, pairso, _, _, _ = timed(sim)
        sim.close()
        fp32d = {"value": round(no * args.steps / elo, 1), "unit": "particle-steps/s",
                 "ms_per_step": round(elo * 1e3 / args.steps, 5), "pair_evals_per_s": round(pairso / elo, 1),
                 "precision": ("binary32 state, binary64 displacements (trajectories bit for bit the oracle's), "
                               "p_enc with binary64 near-contact arguments, binary64 propagation"
                               if other == S.PREC_FP32_FP64NC else
                               "binary32 state and displacements (binary32 Box-Muller); p_enc with binary64 "
                               "near-contact arguments; binary64 propagation; held to the oracle by stage parity")}
        log(f"[bench] other near-contact mode: {fp32d}")
    # pass 2: the same steps with HIP events around every kernel -> kernel durations
    kt, el_ev = {}, None
    if not args.no_timing:
        sim = make(True)
        el_ev, _, _, c0, c1, kt = timed(sim)
        sim.close()
        log(f"[bench] events: {args.steps} steps in {el_ev * 1e3:.1f} ms; kernel times {kt}")

    # dominant kernel and its roofline
    n_keys = 3 * grid[3]
    rec_scale = 2 if cfg["precision"] == S.PREC_FP64 else 1  # 32-byte binary64 records
    per = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kt.items()}
    tot = {k: v[0] for k, v in kt.items()}
    dom = max(tot, key=tot.get) if any(tot.values()) else None
    # the rocprofv3 counts were taken on the default run of this workload
    profiled = (args.workload == "cfg_rad3d" and args.precision == "workload" and args.pair_search == "auto"
                and args.cell == 0.0 and not args.autotune and args.scale == 1.0 and args.eps_cut == 1e-6)

    def hbm_roof(k):
        if per.get(k, 0.0) <= 0.0:
            return None
        nb = algorithmic_bytes(k, n_live, 0.5 * (c0["A"] + c1["A"]), 0.5 * (c0["B"] + c1["B"]), n_keys)
        if nb is None:
            return None
        nb *= rec_scale
        ach = nb / (per[k] * 1e-3) / 1e9
        return {"kernel": k, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(k) if profiled else None,
                "algorithmic_bytes_per_launch": int(nb), "avg_launch_ms": round(per[k], 5),
                "valu_issue": valu_issue(k, per[k]) if profiled else None}

    move_roof = hbm_roof("move")
    roof = angle_step_roofline(per["angles"], profiled) if dom == "angles" else (hbm_roof(dom) if dom else None)

    if args.extras:
        gen.join()
        extras["pair_probs"] = pair_probs_record(10_000_000, 20, 3, I, S)
        extras["ensemble"] = ensemble_record(extras.pop("reps"), S)
        extras["served"] = served_record(extras.pop("trace"), S)

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
        "dtype": "f64" if cfg["precision"] == S.PREC_FP64 else "f32",
        "data": "synthetic",
        "pair_evals_per_s": round(pairs / el, 1),
        "config": {"workload": describe(cfg), "eps_cut": args.eps_cut,
                   "precision": {S.PREC_FP64: "binary64 throughout",
                                 S.PREC_FP32: "binary32 state, pair test and p_enc; binary64 propagation",
                                 S.PREC_FP32_FP64NC: "binary32 state and p_enc, binary64 near-contact arguments and "
                                                     "propagation",
                                 S.PREC_FP32D_FP64NC: "binary32 state, displacements and p_enc, binary64 near-contact "
                                                      "arguments and propagation"}[cfg["precision"]],
                   "particles": len(sp), "r_cut_um": der["rcut"], "cells": grid[:3],
                   "pair_search": {S.PAIRS_BRICKS: "lds-bricks", S.PAIRS_DIRECT: "direct"}[grid[4]],
                   "step_launch": "one hipGraph replay per step",
                   "cell_edge_um": der["cell"],
                   "green2d": args.green2d if dim == 2 else None,
                   **({"unvalidated_tau": True} if args.unvalidated_tau else {}),
                   "handle_creation_s": round(t_create, 3)},
        "autotune": tuned,
        "plain_fp32": plain,
        "other_near_contact_mode": fp32d,
        "roofline": roof,
        "move_roofline": move_roof,
        "kernel_ms_per_step": {k: round(v[0] / max(args.steps, 1), 5) for k, v in kt.items()},
        "cpu_baseline": cpu,
        "ensemble": extras.get("ensemble"),
        "served": extras.get("served"),
        "pair_probs": extras.get("pair_probs"),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
