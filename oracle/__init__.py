"""FP64 CPU oracle for the Green's-function Brownian-dynamics step (arXiv:1107.0270).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It wraps the plain
C implementation in ``gfbd_oracle.c`` through ctypes and shares nothing with the
HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gfbd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

SP_A, SP_B, SP_C, SP_FREE, SP_RESERVED = 0, 1, 2, 3, 4
BC_ABS, BC_REF, BC_RAD = 0, 1, 2
STAT_NAMES = ["pairs", "cand", "overlap", "r0clamp", "picks", "matches", "react", "decay",
              "geminate", "attempts", "bound_hits"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (ISO C99, binary64, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", _LIB_PATH, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


class Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("bc", C.c_int32), ("store_f32", C.c_int32), ("n_terms", C.c_int32),
                ("box", C.c_double * 3), ("dt", C.c_double), ("D", C.c_double * 3), ("sigma", C.c_double),
                ("kappa_a", C.c_double), ("k_off", C.c_double), ("eps_cut", C.c_double), ("rcut", C.c_double),
                ("seed", C.c_uint64), ("replica", C.c_uint32), ("exact2d", C.c_int32), ("keep_dir", C.c_int32)]


PAIR_DT = np.dtype([("i", "<u4"), ("j", "<u4"), ("R", "<f8"), ("R0", "<f8"), ("p", "<f8"),
                    ("draw", "<u4"), ("cand", "<i4")], align=True)
PICK_DT = np.dtype([("i", "<u4"), ("j", "<u4"), ("p", "<f8")], align=True)
MATCH_DT = np.dtype([("i", "<u4"), ("j", "<u4"), ("reacted", "<i4"), ("attempts", "<u4"), ("draw", "<u4"),
                     ("pad", "<u4"), ("Rpp", "<f8"), ("preac", "<f8"), ("cos_theta", "<f8")], align=True)
DISS_DT = np.dtype([("c", "<u4"), ("j", "<u4"), ("decayed", "<i4"), ("recombined", "<i4"),
                    ("attempts", "<u4"), ("draw", "<u4"), ("Rpp", "<f8"), ("preac", "<f8")], align=True)

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    L = C.CDLL(_LIB_PATH)
    d, i, u32, u64, vp = C.c_double, C.c_int, C.c_uint32, C.c_uint64, C.c_void_p
    P = C.POINTER
    sig = {
        "orc_philox4x32_10": (None, [P(u32), P(u32), P(u32)]),
        "orc_u01": (d, [u32]),
        "orc_erfcx": (d, [d]),
        "orc_ierfcx": (None, [d, i, P(d)]),
        "orc_i0e": (d, [d]),
        "orc_erfc_tail_inv": (d, [d, d]),
        "orc_asym_coeffs": (None, [d, i, P(d)]),
        "orc_g3_free": (d, [d, d, d]),
        "orc_g3_abs": (d, [d, d, d]),
        "orc_g3_rad": (d, [d, d, d, d]),
        "orc_penc3": (d, [d, d, d]),
        "orc_preac3": (d, [d, d, d, d]),
        "orc_loss3_abs": (d, [d, d]),
        "orc_loss3_rad": (d, [d, d, d]),
        "orc_prop3_density": (d, [d, d, d]),
        "orc_gamma2": (None, [d, d, d, i, P(d), P(d), P(d)]),
        "orc_g2_bc": (d, [i, d, d, d, d, i]),
        "orc_g2_free": (d, [d, d, d]),
        "orc_penc2": (d, [d, d, d, i]),
        "orc_preac2": (d, [d, d, d, d, i]),
        "orc_prop2_density": (d, [d, d, d, i]),
        "orc_sample_prop": (d, [i, d, d, i, P(u32), P(u32), P(u32), P(u32)]),
        "orc_g2x": (None, [d, d, d, d, P(d)]),
        "orc_m2x": (None, [d, d, d, P(d)]),
        "orc_penc2x": (d, [d, d, d]),
        "orc_preac2x": (d, [d, d, d, d]),
        "orc_sample_prop2x": (d, [d, d, d]),
        "orc_x2_switch": (d, [d]),
        "orc_x2_prop_switch": (d, [d]),
        "orc_first_passage": (u64, [i, P(d), P(d), d, i, i, u32, u32, P(u32), P(u32)]),
        "orc_rcut": (d, [i, i, d, d, d, d, d]),
        "orc_angle3_terms": (i, [d, d, d]),
        "orc_bessel_half": (None, [i, d, P(d), P(d)]),
        "orc_angle3_coef": (None, [i, d, d, d, i, P(d)]),
        "orc_angle3_cdf": (d, [P(d), i, d]),
        "orc_sample_angle3": (d, [d, d, d, d]),
        "orc_bessel_int": (None, [i, d, P(d), P(d)]),
        "orc_angle2_coef": (None, [i, d, d, d, i, P(d)]),
        "orc_angle2_cdf": (d, [P(d), i, d]),
        "orc_sample_angle2": (d, [d, d, d, d]),
        "orc_sim_create": (vp, [P(Params), u64, vp, vp, vp]),
        "orc_sim_destroy": (None, [vp]),
        "orc_sim_step": (None, [vp]),
        "orc_sim_cap": (u64, [vp]),
        "orc_sim_stepno": (u64, [vp]),
        "orc_sim_derived": (None, [vp, P(d)]),
        "orc_sim_state": (None, [vp, vp, vp, vp]),
        "orc_sim_moved": (None, [vp, vp]),
        "orc_sim_set_moved": (None, [vp, vp, vp]),
        "orc_sim_moved_own": (None, [vp, vp]),
        "orc_sim_stats": (None, [vp, P(u64)]),
        "orc_sim_n_pairs": (u64, [vp]),
        "orc_sim_n_picks": (u64, [vp]),
        "orc_sim_n_matches": (u64, [vp]),
        "orc_sim_n_diss": (u64, [vp]),
        "orc_sim_pairs": (None, [vp, vp]),
        "orc_sim_picks": (None, [vp, vp]),
        "orc_sim_matches": (None, [vp, vp]),
        "orc_sim_diss": (None, [vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---- scalar wrappers --------------------------------------------------------

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def u01(x):
    return lib().orc_u01(int(x) & 0xFFFFFFFF)


def erfcx(x):
    return lib().orc_erfcx(float(x))


def ierfcx(x, kmax):
    out = np.zeros(kmax + 2)
    lib().orc_ierfcx(float(x), int(kmax), _dp(out))
    return out


def i0e(x):
    return lib().orc_i0e(float(x))


def erfc_tail_inv(yc, u):
    return lib().orc_erfc_tail_inv(float(yc), float(u))


def asym_coeffs(nu, n):
    out = np.zeros(n + 1)
    lib().orc_asym_coeffs(float(nu), int(n), _dp(out))
    return out


def g3_free(R, R0, tau):
    return lib().orc_g3_free(R, R0, tau)


def g3_abs(R, R0, tau):
    return lib().orc_g3_abs(R, R0, tau)


def g3_rad(R, R0, tau, hh):
    return lib().orc_g3_rad(R, R0, tau, hh)


def penc3(R, R0, tau):
    return lib().orc_penc3(R, R0, tau)


def preac3(R, R0, tau, hh):
    return lib().orc_preac3(R, R0, tau, hh)


def loss3_abs(R0, tau):
    return lib().orc_loss3_abs(R0, tau)


def loss3_rad(R0, tau, hh):
    return lib().orc_loss3_rad(R0, tau, hh)


def prop3_density(Rp, R0, tau):
    return lib().orc_prop3_density(Rp, R0, tau)


def gamma2(R, R0, hh, n):
    ga, gf, gr = np.zeros(n + 1), np.zeros(n + 1), np.zeros(n + 1)
    lib().orc_gamma2(R, R0, hh, n, _dp(ga), _dp(gf), _dp(gr))
    return ga, gf, gr


def g2_bc(kind, R, R0, tau, hh, n):
    return lib().orc_g2_bc(int(kind), R, R0, tau, hh, int(n))


def g2_free(R, R0, tau):
    return lib().orc_g2_free(R, R0, tau)


def penc2(R, R0, tau, n):
    return lib().orc_penc2(R, R0, tau, int(n))


def preac2(R, R0, tau, hh, n):
    return lib().orc_preac2(R, R0, tau, hh, int(n))


def prop2_density(Rp, R0, tau, n):
    return lib().orc_prop2_density(Rp, R0, tau, int(n))


def sample_prop(dim, R0, tau, n_terms, ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    att, hits = C.c_uint32(0), C.c_uint32(0)
    Rp = lib().orc_sample_prop(int(dim), float(R0), float(tau), int(n_terms), c, k, C.byref(att), C.byref(hits))
    return Rp, att.value, hits.value


def g2x(R, R0, tau, hh):
    """Exact 2D radial Green's functions (a^2 g_abs, g_ref, g_rad) by quadrature."""
    out = np.zeros(3)
    lib().orc_g2x(float(R), float(R0), float(tau), float(hh), _dp(out))
    return out


def m2x(R, R0, tau):
    """int_1^R 2 pi R' g(R'|R0) dR' of the absorbing and reflecting functions."""
    out = np.zeros(2)
    lib().orc_m2x(float(R), float(R0), float(tau), _dp(out))
    return out


def penc2x(R, R0, tau):
    return lib().orc_penc2x(float(R), float(R0), float(tau))


def preac2x(R, R0, tau, hh):
    return lib().orc_preac2x(float(R), float(R0), float(tau), float(hh))


def sample_prop2x(R0, tau, u):
    return lib().orc_sample_prop2x(float(R0), float(tau), float(u))


def x2_switch(tau):
    return lib().orc_x2_switch(float(tau))


def x2_prop_switch(tau):
    return lib().orc_x2_prop_switch(float(tau))


def first_passage(dim, xi, xf, tau, levels, c0, step, key, n_terms=12):
    """First contact of a pair by bisection (Appendix): the index lo of the interval
    [lo, lo + 1) * dt / 2^levels, and the midpoint proposals drawn."""
    a = np.zeros(3)
    b = np.zeros(3)
    a[:dim] = np.asarray(xi, dtype=np.float64).reshape(-1)[:dim]
    b[:dim] = np.asarray(xf, dtype=np.float64).reshape(-1)[:dim]
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    att = C.c_uint32(0)
    lo = lib().orc_first_passage(int(dim), _dp(a), _dp(b), float(tau), int(levels), int(n_terms),
                                 int(c0) & 0xFFFFFFFF, int(step) & 0xFFFFFFFF, k, C.byref(att))
    return int(lo), att.value


def angle3_terms(R, R0, tau):
    """Legendre terms kept by the 3D angular propagator."""
    return lib().orc_angle3_terms(float(R), float(R0), float(tau))


def bessel_half(kmax, z):
    """(J, Y): J[k] = J_{k-1/2}(z), Y[k] = Y_{k-1/2}(z) for k = 0 .. kmax."""
    J = np.zeros(kmax + 1)
    Y = np.zeros(kmax + 1)
    lib().orc_bessel_half(int(kmax), float(z), _dp(J), _dp(Y))
    return J, Y


def angle3_coef(kind, R, R0, tau, N=None):
    """Legendre coefficients w_0..w_N of G_ref - G_abs (kind 0) or of the free
    Green's function (kind 1), eq. genericGF3D in units a = 1, D_eff = 1."""
    if N is None:
        N = angle3_terms(R, R0, tau)
    w = np.zeros(N + 1)
    lib().orc_angle3_coef(int(kind), float(R), float(R0), float(tau), int(N), _dp(w))
    return w


def angle3_cdf(w, c):
    """Distribution function of cos Theta given R from the coefficients w."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    return lib().orc_angle3_cdf(_dp(w), len(w) - 1, float(c))


def sample_angle3(R, R0, tau, u):
    """cos Theta drawn from J (G_ref - G_abs) given R by inversion at u."""
    return lib().orc_sample_angle3(float(R), float(R0), float(tau), float(u))


def bessel_int(kmax, z):
    """(J, Y): J[k] = J_{k-1}(z), Y[k] = Y_{k-1}(z) for k = 0 .. kmax."""
    J = np.zeros(kmax + 1)
    Y = np.zeros(kmax + 1)
    lib().orc_bessel_int(int(kmax), float(z), _dp(J), _dp(Y))
    return J, Y


def angle2_coef(kind, R, R0, tau, N=None):
    """Coefficients w_0..w_N of the cos(n theta) series of G_ref - G_abs (kind 0) or of the
    free Green's function (kind 1), eq. genericGF in units a = 1, D_eff = 1."""
    if N is None:
        N = angle3_terms(R, R0, tau)
    w = np.zeros(N + 1)
    lib().orc_angle2_coef(int(kind), float(R), float(R0), float(tau), int(N), _dp(w))
    return w


def angle2_cdf(w, t):
    """Distribution function of |theta| in [0, pi] given R from the coefficients w."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    return lib().orc_angle2_cdf(_dp(w), len(w) - 1, float(t))


def sample_angle2(R, R0, tau, u):
    """|theta| drawn from r (G_ref - G_abs) given R by inversion at u."""
    return lib().orc_sample_angle2(float(R), float(R0), float(tau), float(u))


def rcut(dim, bc, a, Deff, dt, kappa_a, eps):
    return lib().orc_rcut(int(dim), int(bc), a, Deff, dt, kappa_a, eps)


# ---- simulation -------------------------------------------------------------

class OracleSim:
    """The step of Sec. 3 on a slot-indexed state, in FP64."""

    def __init__(self, *, dim, bc, box, dt, D, sigma, kappa_a=0.0, k_off=0.0, eps_cut=1e-3, rcut=0.0,
                 seed=0, replica=0, store_f32=False, n_terms=12, exact2d=False, keep_direction=False, species, pos,
                 partner=None):
        L = lib()
        p = Params()
        p.dim, p.bc, p.store_f32, p.n_terms = int(dim), int(bc), int(bool(store_f32)), int(n_terms)
        p.exact2d = int(bool(exact2d))
        p.keep_dir = int(bool(keep_direction))
        self.keep_direction = bool(keep_direction)
        bx = list(box) + [1.0] * (3 - len(box))
        for k in range(3):
            p.box[k] = float(bx[k])
        Dl = list(D) + [0.0] * (3 - len(D))
        for k in range(3):
            p.D[k] = float(Dl[k])
        p.dt, p.sigma, p.kappa_a, p.k_off = float(dt), float(sigma), float(kappa_a), float(k_off)
        p.eps_cut, p.rcut, p.seed, p.replica = float(eps_cut), float(rcut), int(seed), int(replica)
        self._p = p
        self.dim = int(dim)
        sp = np.ascontiguousarray(species, dtype=np.int32)
        ps = np.ascontiguousarray(pos, dtype=np.float64).reshape(len(sp), self.dim)
        pt = None if partner is None else np.ascontiguousarray(partner, dtype=np.uint32)
        self.n = len(sp)
        self._h = L.orc_sim_create(C.byref(p), self.n, sp.ctypes.data, ps.ctypes.data,
                                   None if pt is None else pt.ctypes.data)
        self._keep = (sp, ps, pt)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_sim_destroy(h)
            self._h = None

    def step(self, n=1):
        for _ in range(n):
            lib().orc_sim_step(self._h)

    @property
    def stepno(self):
        return int(lib().orc_sim_stepno(self._h))

    def derived(self):
        out = np.zeros(6)
        lib().orc_sim_derived(self._h, _dp(out))
        return dict(zip(["Deff", "tau", "hh", "rcut", "a", "p_uni"], out.tolist()))

    def state(self):
        sp = np.zeros(self.n, np.int32)
        pos = np.zeros((self.n, self.dim))
        pt = np.zeros(self.n, np.uint32)
        lib().orc_sim_state(self._h, sp.ctypes.data, pos.ctypes.data, pt.ctypes.data)
        return sp, pos, pt

    def moved(self):
        pos = np.zeros((self.n, self.dim))
        lib().orc_sim_moved(self._h, pos.ctypes.data)
        return pos

    def set_moved(self, pos, disp):
        """Stage parity: the next step takes these post-move positions and displacements ((n, dim)
        each, by slot) in place of its own move; its own move is kept (moved_own)."""
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(self.n, self.dim)
        disp = np.ascontiguousarray(disp, dtype=np.float64).reshape(self.n, self.dim)
        lib().orc_sim_set_moved(self._h, pos.ctypes.data, disp.ctypes.data)
        self._given = (pos, disp)

    def moved_own(self):
        pos = np.zeros((self.n, self.dim))
        lib().orc_sim_moved_own(self._h, pos.ctypes.data)
        return pos

    def stats(self):
        out = (C.c_uint64 * len(STAT_NAMES))()
        lib().orc_sim_stats(self._h, out)
        return dict(zip(STAT_NAMES, [int(x) for x in out]))

    def _log(self, count_fn, get_fn, dt):
        n = int(count_fn(self._h))
        a = np.zeros(n, dtype=dt)
        if n:
            get_fn(self._h, a.ctypes.data)
        return a

    def pairs(self):
        L = lib()
        return self._log(L.orc_sim_n_pairs, L.orc_sim_pairs, PAIR_DT)

    def picks(self):
        L = lib()
        return self._log(L.orc_sim_n_picks, L.orc_sim_picks, PICK_DT)

    def matches(self):
        L = lib()
        return self._log(L.orc_sim_n_matches, L.orc_sim_matches, MATCH_DT)

    def dissociations(self):
        L = lib()
        return self._log(L.orc_sim_n_diss, L.orc_sim_diss, DISS_DT)
