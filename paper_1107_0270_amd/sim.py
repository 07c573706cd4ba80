"""Thin ctypes binding of the C-ABI in include/gfbd.h (argument marshalling only).

Every step of the simulation runs in the HIP kernels of ``libgfbd.so``; this module
only converts Python/numpy arguments and raises on error codes.  It refuses to run
if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgfbd.so")

SIM_OK, SIM_EINVAL, SIM_ENOMEM, SIM_EDEVICE, SIM_ESTATE, SIM_EUNSUPPORTED, SIM_ECAPACITY = 0, -1, -2, -3, -4, -5, -6
SP_A, SP_B, SP_C, SP_FREE, SP_RESERVED = 0, 1, 2, 3, 4
BC_ABSORBING, BC_REFLECTING, BC_RADIATION = 0, 1, 2
PREC_FP64, PREC_FP32, PREC_FP32_FP64NC, PREC_FP32D_FP64NC = 0, 1, 2, 3
PAIRS_AUTO, PAIRS_BRICKS, PAIRS_DIRECT = 0, 1, 2
G2_EXPANSION, G2_EXACT = 0, 1
F_UNVALIDATED_TAU, F_KEEP_DIRECTION = 1, 2
(READ_POS, READ_SPECIES, READ_PARTNER, READ_COUNTS, READ_STATS, READ_STATS_SUM, READ_DERIVED, READ_DBG_MOVED,
 READ_DBG_PAIRS, READ_DBG_PICKS, READ_DBG_MATCHES, READ_DBG_DISS, READ_DBG_CELLS, READ_TIMING, READ_GRID,
 READ_DBG_DISP) = range(16)
STAT_NAMES = ["pairs", "cand", "overlap", "r0clamp", "picks", "matches", "react", "decay", "geminate",
              "attempts", "bound_hits", "near", "lds_fallback"]
KERNEL_NAMES = ["move", "scan", "scatter", "pairs", "eval", "select_a", "select_b", "events", "angles"]

PAIR_DT = np.dtype([("i", "<u4"), ("j", "<u4"), ("R", "<f8"), ("R0", "<f8"), ("p", "<f8"),
                    ("draw", "<u4"), ("cand", "<i4")], align=True)
PICK_DT = np.dtype([("i", "<u4"), ("j", "<u4"), ("p", "<f8")], align=True)
MATCH_DT = np.dtype([("i", "<u4"), ("j", "<u4"), ("reacted", "<i4"), ("attempts", "<u4"), ("draw", "<u4"),
                     ("pad", "<u4"), ("Rpp", "<f8"), ("preac", "<f8"), ("cos_theta", "<f8")], align=True)
DISS_DT = np.dtype([("c", "<u4"), ("j", "<u4"), ("decayed", "<i4"), ("recombined", "<i4"),
                    ("attempts", "<u4"), ("draw", "<u4"), ("Rpp", "<f8"), ("preac", "<f8")], align=True)


class SimSpecies(C.Structure):
    _fields_ = [("D", C.c_double)]


class SimReaction(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32), ("c", C.c_int32), ("bc", C.c_int32),
                ("sigma", C.c_double), ("kappa", C.c_double), ("k_off", C.c_double)]


class SimReplica(C.Structure):
    _fields_ = [("n", C.c_uint64), ("species", C.c_void_p), ("pos", C.c_void_p), ("partner", C.c_void_p),
                ("box", C.c_double * 3), ("kappa", C.c_double), ("replica", C.c_uint32), ("step", C.c_uint32)]


class SimConfig(C.Structure):
    _fields_ = [("dim", C.c_int32), ("precision", C.c_int32), ("box", C.c_double * 3), ("dt", C.c_double),
                ("seed", C.c_uint64), ("replica", C.c_uint32), ("n_terms", C.c_int32), ("eps_cut", C.c_double),
                ("rcut", C.c_double), ("cell", C.c_double), ("pair_search", C.c_int32), ("n_species", C.c_int32),
                ("species", C.POINTER(SimSpecies)), ("n_reactions", C.c_int32),
                ("reactions", C.POINTER(SimReaction)), ("debug", C.c_uint32), ("timing", C.c_uint32),
                ("debug_cap", C.c_uint64), ("hip_stream", C.c_void_p), ("green2d", C.c_int32),
                ("pair_blocks", C.c_int32), ("event_blocks", C.c_int32), ("flags", C.c_uint32)]


_hip_rt = None


def hip_runtime():
    """The HIP runtime libgfbd.so is linked against (device buffers for sim_eval_pairs)."""
    global _hip_rt
    if _hip_rt is None:
        lib()
        h = C.CDLL("libamdhip64.so.7")
        h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        h.hipFree.argtypes = [C.c_void_p]
        h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        h.hipDeviceSynchronize.argtypes = []
        _hip_rt = h
    return _hip_rt


class DeviceBuffer:
    """A plain device allocation of the library's HIP runtime."""

    def __init__(self, nbytes):
        self.nbytes = int(nbytes)
        p = C.c_void_p()
        if hip_runtime().hipMalloc(C.byref(p), self.nbytes) != 0:
            raise MemoryError(f"hipMalloc of {self.nbytes} bytes failed")
        self.ptr = p.value

    def upload(self, a):
        a = np.ascontiguousarray(a)
        assert a.nbytes <= self.nbytes
        if hip_runtime().hipMemcpy(self.ptr, a.ctypes.data, a.nbytes, 1) != 0:  # host to device
            raise RuntimeError("hipMemcpy to the device failed")

    def download(self, a):
        assert a.nbytes <= self.nbytes and a.flags["C_CONTIGUOUS"]
        if hip_runtime().hipMemcpy(a.ctypes.data, self.ptr, a.nbytes, 2) != 0:  # device to host
            raise RuntimeError("hipMemcpy from the device failed")
        return a

    def free(self):
        if self.ptr:
            hip_runtime().hipFree(self.ptr)
            self.ptr = None


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gfbd error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libgfbd.so; raise if it was not built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python -m paper_1107_0270_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, u64, u32, i32 = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int32
    L.sim_create.argtypes = [C.POINTER(SimConfig), u64, vp, vp, vp, C.POINTER(vp)]
    L.sim_create.restype = C.c_int
    L.sim_batch_create.argtypes = [C.POINTER(SimConfig), u32, C.POINTER(SimReplica), C.POINTER(vp)]
    L.sim_batch_create.restype = C.c_int
    L.sim_pool_create.argtypes = [C.POINTER(SimConfig), u64, u64, u32, C.POINTER(vp)]
    L.sim_pool_create.restype = C.c_int
    L.sim_pool_admit.argtypes = [vp, C.POINTER(SimReplica), C.POINTER(u32)]
    L.sim_pool_admit.restype = C.c_int
    L.sim_pool_retire.argtypes = [vp, u32]
    L.sim_pool_retire.restype = C.c_int
    L.sim_pool_read.argtypes = [vp, u32, C.c_int, vp, u64, C.POINTER(u64)]
    L.sim_pool_read.restype = C.c_int
    L.sim_step.argtypes = [vp, u32]
    L.sim_step.restype = C.c_int
    L.sim_step_async.argtypes = [vp, u32]
    L.sim_step_async.restype = C.c_int
    L.sim_sync.argtypes = [vp]
    L.sim_sync.restype = C.c_int
    L.sim_read.argtypes = [vp, C.c_int, vp, u64, C.POINTER(u64)]
    L.sim_read.restype = C.c_int
    L.sim_load_state.argtypes = [vp, u64, vp, vp, vp]
    L.sim_load_state.restype = C.c_int
    L.sim_eval_pairs.argtypes = [vp, u64, vp, vp, vp, vp]
    L.sim_eval_pairs.restype = C.c_int
    L.sim_eval_pairs_noalloc.argtypes = [C.POINTER(SimConfig), u64, vp, vp, vp, vp]
    L.sim_eval_pairs_noalloc.restype = C.c_int
    L.sim_eval_propagator.argtypes = [vp, u64, vp, u32, C.c_int, vp, vp]
    L.sim_eval_propagator.restype = C.c_int
    L.sim_eval_first_passage.argtypes = [vp, u64, vp, vp, C.c_int32, u32, vp, vp]
    L.sim_eval_first_passage.restype = C.c_int
    L.sim_eval_angle.argtypes = [vp, u64, vp, vp, vp, vp]
    L.sim_eval_angle.restype = C.c_int
    L.sim_destroy.argtypes = [vp]
    L.sim_destroy.restype = C.c_int
    L.sim_last_error.argtypes = [vp]
    L.sim_last_error.restype = C.c_char_p
    _lib = L
    return L


def _fill_replica(rep, rd, dim, kappa0, default_replica):
    """Fill a SimReplica from a dict (species, pos, box; optional kappa, replica, step, partner).
    Returns the arrays the struct points into (to be kept alive by the caller)."""
    sp = np.ascontiguousarray(rd["species"], dtype=np.int32)
    ps = np.ascontiguousarray(rd["pos"], dtype=np.float64).ravel()
    if ps.size != dim * sp.size:
        raise ValueError("pos must hold n * dim values")
    pt = None if rd.get("partner") is None else np.ascontiguousarray(rd["partner"], dtype=np.uint32)
    bx = list(rd["box"]) if np.ndim(rd["box"]) else [float(rd["box"])] * dim
    bx = bx + [1.0] * (3 - len(bx))
    rep.n = sp.size
    rep.species, rep.pos = sp.ctypes.data, ps.ctypes.data
    rep.partner = None if pt is None else pt.ctypes.data
    for k in range(3):
        rep.box[k] = float(bx[k])
    rep.kappa = float(rd.get("kappa", kappa0))
    rep.replica = int(rd.get("replica", default_replica))
    rep.step = int(rd.get("step", 0))
    return (sp, ps, pt)


class Sim:
    """One simulation handle on the GPU (see include/gfbd.h for the semantics)."""

    def __init__(self, *, dim, box, dt, D, sigma, bc, species, pos, kappa=0.0, k_off=0.0,
                 precision=PREC_FP32_FP64NC, seed=0, replica=0, n_terms=12, eps_cut=1e-3, rcut=0.0, cell=0.0,
                 pair_search=PAIRS_AUTO, partner=None, debug=False, timing=False, debug_cap=0, stream=None,
                 green2d=G2_EXPANSION, pair_blocks=0, event_blocks=0, flags=0):
        self._config(dim=dim, box=box, dt=dt, D=D, sigma=sigma, bc=bc, species=species, pos=pos, kappa=kappa,
                     k_off=k_off, precision=precision, seed=seed, replica=replica, n_terms=n_terms, eps_cut=eps_cut,
                     rcut=rcut, cell=cell, pair_search=pair_search, debug=debug, timing=timing, debug_cap=debug_cap,
                     stream=stream, green2d=green2d, pair_blocks=pair_blocks, event_blocks=event_blocks, flags=flags)
        L = lib()
        cfg = self.cfg
        sp = np.ascontiguousarray(species, dtype=np.int32)
        self.n = len(sp)
        ps = np.ascontiguousarray(pos, dtype=np.float64).ravel()
        if self.dim in (2, 3) and ps.size != self.n * self.dim:
            raise ValueError("pos must hold n * dim values")
        pt = None if partner is None else np.ascontiguousarray(partner, dtype=np.uint32)
        h = C.c_void_p()
        rc = L.sim_create(C.byref(cfg), self.n, sp.ctypes.data, ps.ctypes.data,
                          None if pt is None else pt.ctypes.data, C.byref(h))
        if rc != SIM_OK:
            raise SimError(rc, L.sim_last_error(None).decode())
        self._h = h
        self.slot_base = [0]

    def _config(self, *, dim, box, dt, D, sigma, bc, species, pos, kappa=0.0, k_off=0.0,
                precision=PREC_FP32_FP64NC, seed=0, replica=0, n_terms=12, eps_cut=1e-3, rcut=0.0, cell=0.0,
                pair_search=PAIRS_AUTO, debug=False, timing=False, debug_cap=0, stream=None, green2d=G2_EXPANSION,
                pair_blocks=0, event_blocks=0, flags=0):
        cfg = SimConfig()
        cfg.dim, cfg.precision = int(dim), int(precision)
        bx = list(box) if np.ndim(box) else [float(box)] * int(dim)
        bx = bx + [1.0] * (3 - len(bx))
        for k in range(3):
            cfg.box[k] = float(bx[k])
        cfg.dt, cfg.seed, cfg.replica, cfg.n_terms = float(dt), int(seed), int(replica), int(n_terms)
        cfg.eps_cut, cfg.rcut, cfg.cell = float(eps_cut), float(rcut), float(cell)
        cfg.pair_search = int(pair_search)
        Dl = list(D)
        if len(Dl) == 2:
            Dl.append(Dl[0] * Dl[1] / (Dl[0] + Dl[1]))
        self._species = (SimSpecies * 3)(*[SimSpecies(float(x)) for x in Dl])
        self._reaction = (SimReaction * 1)(SimReaction(0, 1, 2, int(bc), float(sigma), float(kappa), float(k_off)))
        cfg.n_species, cfg.species = 3, self._species
        cfg.n_reactions, cfg.reactions = 1, self._reaction
        cfg.debug, cfg.timing, cfg.debug_cap = int(bool(debug)), int(bool(timing)), int(debug_cap)
        cfg.hip_stream = stream
        cfg.green2d = int(green2d)
        cfg.pair_blocks, cfg.event_blocks = int(pair_blocks), int(event_blocks)
        cfg.flags = int(flags)
        self.cfg = cfg
        self.dim = int(dim)

    @classmethod
    def batch(cls, replicas, **shared):
        """A handle stepping independent replicas together (sim_batch_create).  ``replicas`` is a
        list of dicts with ``species``, ``pos``, ``box`` and optional ``kappa``, ``replica``, ``step``
        and ``partner`` (replica-local); ``shared`` takes the Sim keywords common to all (``dim``,
        default 3).
        Slots of replica r follow those of replicas 0..r-1 in every read (``self.slot_base``)."""
        L = lib()
        first = replicas[0]
        self = cls.__new__(cls)
        shared = dict(shared)
        kappa0 = shared.pop("kappa", 0.0)
        # a config exactly as the single-system constructor builds it, with replica 0's values
        cfg_self = cls.__new__(cls)
        dim = int(shared.pop("dim", 3))
        cls._config(cfg_self, dim=dim, box=first["box"], species=np.zeros(1, np.int32), pos=np.zeros(dim),
                    kappa=first.get("kappa", kappa0), **shared)
        self.cfg, self._species, self._reaction = cfg_self.cfg, cfg_self._species, cfg_self._reaction
        self.dim = dim
        keep, reps = [], (SimReplica * len(replicas))()
        bases, n = [], 0
        for r, rd in enumerate(replicas):
            keep.append(_fill_replica(reps[r], rd, dim, kappa0, r))
            bases.append(n)
            n += reps[r].n
        h = C.c_void_p()
        rc = L.sim_batch_create(C.byref(self.cfg), len(replicas), reps, C.byref(h))
        if rc != SIM_OK:
            raise SimError(rc, L.sim_last_error(None).decode())
        self._h, self.n, self.slot_base = h, n, bases
        return self

    # ---- calls ------------------------------------------------------------
    def _check(self, rc):
        if rc != SIM_OK:
            raise SimError(rc, lib().sim_last_error(self._h).decode())

    def step(self, n=1):
        self._check(lib().sim_step(self._h, int(n)))

    def step_async(self, n=1):
        """sim_step_async: enqueue n steps on the handle's stream and return."""
        self._check(lib().sim_step_async(self._h, int(n)))

    def sync(self):
        """sim_sync: wait for the enqueued steps (raises on a per-step buffer overflow)."""
        self._check(lib().sim_sync(self._h))

    def load_state(self, step, species, pos, partner=None):
        sp = np.ascontiguousarray(species, dtype=np.int32)
        ps = np.ascontiguousarray(pos, dtype=np.float64).reshape(self.n, self.dim)
        pt = None if partner is None else np.ascontiguousarray(partner, dtype=np.uint32)
        self._check(lib().sim_load_state(self._h, int(step), sp.ctypes.data, ps.ctypes.data,
                                         None if pt is None else pt.ctypes.data))

    def close(self):
        if getattr(self, "_h", None):
            lib().sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _read(self, what, out):
        w = C.c_uint64(0)
        self._check(lib().sim_read(self._h, what, out.ctypes.data, out.nbytes, C.byref(w)))
        return w.value

    def _read_log(self, what, dt):
        cap = int(self.cfg.debug_cap) or (1 << 20)
        out = np.empty(cap, dtype=dt)
        w = self._read(what, out)
        return out[: w // dt.itemsize].copy()

    # ---- reads ------------------------------------------------------------
    def positions(self):
        out = np.zeros((self.n, self.dim))
        self._read(READ_POS, out)
        return out

    def species(self):
        out = np.zeros(self.n, np.int32)
        self._read(READ_SPECIES, out)
        return out

    def partners(self):
        out = np.zeros(self.n, np.uint32)
        self._read(READ_PARTNER, out)
        return out

    def state(self):
        return self.species(), self.positions(), self.partners()

    def counts(self):
        out = np.zeros(5, np.int64)
        self._read(READ_COUNTS, out)
        return dict(zip(["A", "B", "C", "FREE", "RESERVED"], out.tolist()))

    def stats(self, total=False):
        out = np.zeros(len(STAT_NAMES), np.uint64)
        self._read(READ_STATS_SUM if total else READ_STATS, out)
        return dict(zip(STAT_NAMES, [int(x) for x in out]))

    def derived(self):
        out = np.zeros(8)
        self._read(READ_DERIVED, out)
        return dict(zip(["Deff", "tau", "hh", "rcut", "a", "p_uni", "cell", "step"], out.tolist()))

    def eval_pairs(self, R, R0, penc=True, preac=True):
        """p_enc and p_reac of (R, R0) pairs on the device (sim_eval_pairs).  R and R0 are host
        arrays; they are copied to device buffers and the results back."""
        R = np.ascontiguousarray(R, dtype=np.float64)
        R0 = np.ascontiguousarray(R0, dtype=np.float64)
        if R.shape != R0.shape or R.ndim != 1:
            raise ValueError("R and R0 must be 1-D and of equal length")
        n = R.size
        bufs = [DeviceBuffer(8 * n) for _ in range(4)]
        try:
            bufs[0].upload(R)
            bufs[1].upload(R0)
            self.eval_pairs_device(n, bufs[0].ptr, bufs[1].ptr, bufs[2].ptr if penc else None,
                                   bufs[3].ptr if preac else None)
            out = []
            for want, b in ((penc, bufs[2]), (preac, bufs[3])):
                out.append(b.download(np.empty(n, np.float64)) if want else None)
            return tuple(out)
        finally:
            for b in bufs:
                b.free()

    def eval_propagator(self, R0, step, wave=True):
        """R'' draws for the given R0 (sim_eval_propagator); returns (Rpp, attempts) as numpy arrays."""
        R0 = np.ascontiguousarray(R0, dtype=np.float64)
        n = R0.size
        b_r0, b_r, b_a = DeviceBuffer(8 * n), DeviceBuffer(8 * n), DeviceBuffer(4 * n)
        try:
            b_r0.upload(R0)
            self._check(lib().sim_eval_propagator(self._h, n, b_r0.ptr, int(step), int(bool(wave)), b_r.ptr, b_a.ptr))
            return b_r.download(np.empty(n, np.float64)), b_a.download(np.empty(n, np.uint32))
        finally:
            for b in (b_r0, b_r, b_a):
                b.free()

    def eval_propagator_device(self, n, R0, step, wave, Rpp, attempts):
        """sim_eval_propagator on caller-owned device pointers (ints; attempts may be None)."""
        self._check(lib().sim_eval_propagator(self._h, int(n), R0, int(step), int(bool(wave)), Rpp, attempts))

    def eval_first_passage(self, xi, xf, levels, step=0):
        """First contact of pairs by bisection (sim_eval_first_passage): xi, xf are (n, 3)
        separations in units of a before and after the step; returns (lo, attempts), the contact
        lying in [lo, lo + 1) * dt / 2^levels."""
        xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, 3)
        xf = np.ascontiguousarray(xf, dtype=np.float64).reshape(-1, 3)
        if xi.shape != xf.shape:
            raise ValueError("xi and xf differ in shape")
        n = xi.shape[0]
        b_i, b_f, b_lo, b_a = DeviceBuffer(24 * n), DeviceBuffer(24 * n), DeviceBuffer(8 * n), DeviceBuffer(4 * n)
        try:
            b_i.upload(xi)
            b_f.upload(xf)
            self._check(lib().sim_eval_first_passage(self._h, n, b_i.ptr, b_f.ptr, int(levels), int(step), b_lo.ptr,
                                                     b_a.ptr))
            return b_lo.download(np.empty(n, np.uint64)), b_a.download(np.empty(n, np.uint32))
        finally:
            for b in (b_i, b_f, b_lo, b_a):
                b.free()

    def eval_first_passage_device(self, n, xi, xf, levels, step, lo, attempts):
        """sim_eval_first_passage on caller-owned device pointers (ints; attempts may be None)."""
        self._check(lib().sim_eval_first_passage(self._h, int(n), xi, xf, int(levels), int(step), lo, attempts))

    def eval_angle(self, R, R0, u):
        """Angles of propagated pairs (sim_eval_angle): cos Theta (3D handles) or |theta| in
        [0, pi] (2D handles); R, R0 the new and old separations in units of a, u the uniforms."""
        R = np.ascontiguousarray(R, dtype=np.float64).ravel()
        R0 = np.ascontiguousarray(R0, dtype=np.float64).ravel()
        u = np.ascontiguousarray(u, dtype=np.float64).ravel()
        if not (R.size == R0.size == u.size):
            raise ValueError("R, R0 and u differ in length")
        n = R.size
        bufs = [DeviceBuffer(8 * n) for _ in range(4)]
        try:
            for b, a in zip(bufs, (R, R0, u)):
                b.upload(a)
            self._check(lib().sim_eval_angle(self._h, n, bufs[0].ptr, bufs[1].ptr, bufs[2].ptr, bufs[3].ptr))
            return bufs[3].download(np.empty(n))
        finally:
            for b in bufs:
                b.free()

    def eval_angle_device(self, n, R, R0, u, out):
        """sim_eval_angle on caller-owned device pointers (ints)."""
        self._check(lib().sim_eval_angle(self._h, int(n), R, R0, u, out))

    def eval_pairs_device(self, n, R, R0, penc, preac):
        """sim_eval_pairs on caller-owned device pointers (ints or None)."""
        self._check(lib().sim_eval_pairs(self._h, int(n), R, R0, penc, preac))

    def grid(self):
        """Cells per edge x, y, z, total cells, pair-search kernel (PAIRS_BRICKS or PAIRS_DIRECT)."""
        out = np.zeros(5, np.int64)
        self._read(READ_GRID, out)
        return out.tolist()

    def kernel_times(self):
        out = np.zeros(len(KERNEL_NAMES), dtype=np.dtype([("ms", "<f8"), ("launches", "<u8")]))
        self._read(READ_TIMING, out)
        return {k: (float(r["ms"]), int(r["launches"])) for k, r in zip(KERNEL_NAMES, out)}

    def dbg_moved(self):
        out = np.zeros((self.n, self.dim))
        self._read(READ_DBG_MOVED, out)
        return out

    def dbg_disp(self):
        out = np.zeros((self.n, self.dim))
        self._read(READ_DBG_DISP, out)
        return out

    def dbg_cells(self):
        out = np.zeros(self.n, np.uint32)
        self._read(READ_DBG_CELLS, out)
        return out

    def dbg_pairs(self):
        return self._read_log(READ_DBG_PAIRS, PAIR_DT)

    def dbg_picks(self):
        return self._read_log(READ_DBG_PICKS, PICK_DT)

    def dbg_matches(self):
        return self._read_log(READ_DBG_MATCHES, MATCH_DT)

    def dbg_diss(self):
        return self._read_log(READ_DBG_DISS, DISS_DT)


class Pool(Sim):
    """Continuous batching (sim_pool_create): systems join (``admit``) and leave (``retire``)
    between steps; ``step`` advances every member.  ``box`` is any valid box of the shared
    configuration (members bring their own); the other keywords are those of Sim."""

    def __init__(self, *, dim, box, slot_cap, cell_cap=None, rep_cap=4096, kappa=0.0, **shared):
        self._config(dim=dim, box=box, species=np.zeros(1, np.int32), pos=np.zeros(dim), kappa=kappa, **shared)
        self.kappa = float(kappa)
        cell_cap = slot_cap if cell_cap is None else cell_cap
        h = C.c_void_p()
        L = lib()
        rc = L.sim_pool_create(C.byref(self.cfg), int(slot_cap), int(cell_cap), int(rep_cap), C.byref(h))
        if rc != SIM_OK:
            raise SimError(rc, L.sim_last_error(None).decode())
        self._h, self.n, self.slot_base = h, int(slot_cap), [0]
        self.members = {}

    def admit(self, species, pos, box, kappa=None, replica=0, step=0, partner=None):
        """Add a system; returns its member entry.  Raises SimError (code SIM_ECAPACITY when
        there is no room: nothing changed)."""
        rep = SimReplica()
        rd = dict(species=species, pos=pos, box=box, replica=replica, step=step, partner=partner)
        if kappa is not None:
            rd["kappa"] = kappa
        keep = _fill_replica(rep, rd, self.dim, self.kappa, replica)
        m = C.c_uint32(0)
        self._check(lib().sim_pool_admit(self._h, C.byref(rep), C.byref(m)))
        del keep
        self.members[m.value] = rep.n
        return m.value

    def try_admit(self, *args, **kw):
        """admit, or None when the pool has no room."""
        try:
            return self.admit(*args, **kw)
        except SimError as e:
            if e.code == SIM_ECAPACITY:
                return None
            raise

    def retire(self, member):
        self._check(lib().sim_pool_retire(self._h, int(member)))
        self.members.pop(member, None)

    def _read_member(self, member, what, out):
        w = C.c_uint64(0)
        self._check(lib().sim_pool_read(self._h, int(member), what, out.ctypes.data, out.nbytes, C.byref(w)))
        return out

    def member_state(self, member):
        """(species, positions, partners) of a member, in its own slot order."""
        n = self.members[member]
        sp = self._read_member(member, READ_SPECIES, np.zeros(n, np.int32))
        pos = self._read_member(member, READ_POS, np.zeros((n, self.dim)))
        pt = self._read_member(member, READ_PARTNER, np.zeros(n, np.uint32))
        return sp, pos, pt

    def member_counts(self, member):
        out = self._read_member(member, READ_COUNTS, np.zeros(5, np.int64))
        return dict(zip(["A", "B", "C", "FREE", "RESERVED"], out.tolist()))


def eval_pairs_noalloc(R, R0, *, dim, dt, D, sigma, bc, kappa=0.0, precision=PREC_FP32_FP64NC, n_terms=12, **kw):
    """sim_eval_pairs_noalloc: p_enc and p_reac of (R, R0) pairs for a system given by its
    configuration (no handle), on the null stream.  R and R0 are host arrays, copied to device
    buffers and the results back after the device has finished."""
    holder = Sim.__new__(Sim)
    Sim._config(holder, dim=dim, box=kw.pop("box", 1.0), dt=dt, D=D, sigma=sigma, bc=bc, kappa=kappa,
                species=np.zeros(1, np.int32), pos=np.zeros(dim), precision=precision, n_terms=n_terms, **kw)
    R = np.ascontiguousarray(R, dtype=np.float64)
    R0 = np.ascontiguousarray(R0, dtype=np.float64)
    n = R.size
    bufs = [DeviceBuffer(8 * n) for _ in range(4)]
    try:
        bufs[0].upload(R)
        bufs[1].upload(R0)
        L = lib()
        rc = L.sim_eval_pairs_noalloc(C.byref(holder.cfg), n, bufs[0].ptr, bufs[1].ptr, bufs[2].ptr, bufs[3].ptr)
        if rc != SIM_OK:
            raise SimError(rc, L.sim_last_error(None).decode())
        if hip_runtime().hipDeviceSynchronize() != 0:
            raise RuntimeError("hipDeviceSynchronize failed")
        return bufs[2].download(np.empty(n, np.float64)), bufs[3].download(np.empty(n, np.float64))
    finally:
        for b in bufs:
            b.free()

