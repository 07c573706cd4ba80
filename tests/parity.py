"""Lock-step comparison of the HIP library (through its C-ABI) with the oracle.

Both sides start from the same seeded state and take the same steps.  After every
step the stage logs are compared: post-move positions, the pair list within
r_cut, p_enc and the Bernoulli draws, the A-side picks, the matched pairs (new
radius, p_reac, reaction flag), the dissociations, and the final state.  A
decision may legitimately differ only where the draw lies within 1e-6 of the
probability; such steps are counted, and the GPU is then reloaded with the
oracle's state (oracle -> GPU only) so the comparison can go on.

In lock-step mode (for a mode whose move is not bit-identical to the oracle's,
the plain binary32 one) positions within pos_tol are accepted and the GPU is
reloaded with the oracle's state after every step that differs, so each step
is compared from identical states; such reloads are counted apart.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle as O
from paper_1107_0270_amd import sim as S

NEAR = 1e-6


@dataclasses.dataclass
class Report:
    steps: int = 0
    pairs: int = 0
    cand: int = 0
    matches: int = 0
    reactions: int = 0
    decays: int = 0
    max_dpos: float = 0.0
    max_dp: float = 0.0
    max_dRpp: float = 0.0
    max_dpreac: float = 0.0
    max_dcos: float = 0.0
    angles: int = 0
    pair_set_mismatch: int = 0
    pair_set_near_cut: int = 0
    draw_mismatch: int = 0
    near_decisions: int = 0
    unexplained: int = 0
    resyncs: int = 0
    pos_resyncs: int = 0
    max_dmove: float = 0.0
    notes: list = dataclasses.field(default_factory=list)


def make_pair(*, dim, bc, box, dt, D, sigma, kappa, k_off, precision, species, pos, partner=None, seed=0,
              n_terms=12, eps_cut=1e-3, rcut=0.0, cell=0.0, debug_cap=1 << 21, pair_search=S.PAIRS_AUTO, exact2d=False,
              keep_direction=False):
    gpu = S.Sim(dim=dim, box=box, dt=dt, D=D, sigma=sigma, bc=bc, kappa=kappa, k_off=k_off, precision=precision,
                seed=seed, n_terms=n_terms, eps_cut=eps_cut, rcut=rcut, cell=cell, species=species, pos=pos,
                partner=partner, debug=True, debug_cap=debug_cap, pair_search=pair_search,
                green2d=S.G2_EXACT if exact2d else S.G2_EXPANSION, flags=S.F_KEEP_DIRECTION if keep_direction else 0)
    if pair_search != S.PAIRS_AUTO and min(gpu.grid()[:dim]) >= 3:
        assert gpu.grid()[4] == pair_search
    orc = O.OracleSim(dim=dim, bc=bc, box=[box] * dim, dt=dt, D=D, sigma=sigma, kappa_a=kappa, k_off=k_off,
                      eps_cut=eps_cut, rcut=rcut, seed=seed, store_f32=precision != S.PREC_FP64, n_terms=n_terms,
                      exact2d=exact2d, keep_direction=keep_direction, species=species, pos=pos, partner=partner)
    return gpu, orc


def _near(draw, p, p_tol):
    """True where the uniform (w + 1/2) 2^-32 of Philox word w lies within the tolerance of p, the
    only place where the two sides may legitimately take different Bernoulli decisions."""
    u = (draw.astype(np.float64) + 0.5) * 2.0 ** -32
    return np.abs(u - p) < max(NEAR, 2 * p_tol)


def _key(a, b):
    return (a.astype(np.uint64) << np.uint64(32)) | b.astype(np.uint64)


def compare_step(gpu, orc, rep: Report, *, p_tol, pos_tol, box, rcut, sp_before, lockstep=False, stage=False):
    """Advance both sides one step and compare; returns True if the states agree afterwards.
    stage: stage parity (the oracle takes the GPU's post-move positions and displacements and
    runs every later stage on them; the move itself is compared with the oracle's own)."""
    gpu.step()
    live = sp_before <= O.SP_C
    if stage:
        gm, gd = gpu.dbg_moved(), gpu.dbg_disp()
        orc.set_moved(np.where(np.isnan(gm), 0.0, gm), np.where(np.isnan(gd), 0.0, gd))
        orc.step()
        om = orc.moved_own()
    else:
        orc.step()
        gm, om = gpu.dbg_moved(), orc.moved()
    rep.steps += 1
    # 1. move
    if live.any():
        d = np.abs(gm[live] - om[live])
        d = np.minimum(d, box - d)
        if not stage:  # in stage parity the later stages start from the GPU's move
            rep.max_dpos = max(rep.max_dpos, float(d.max()))
        rep.max_dmove = max(rep.max_dmove, float(d.max()))
    # 2.-3. pairs, p_enc, draws, candidates
    gp, op = gpu.dbg_pairs(), orc.pairs()
    rep.pairs += len(op)
    rep.cand += int(op["cand"].sum())
    gk, ok = _key(gp["i"], gp["j"]), _key(op["i"], op["j"])
    gi, oi = np.argsort(gk), np.argsort(ok)
    gp, op, gk, ok = gp[gi], op[oi], gk[gi], ok[oi]
    if len(gp) != gpu.stats()["pairs"]:
        raise AssertionError(f"GPU pair log truncated: {len(gp)} of {gpu.stats()['pairs']} (raise debug_cap)")
    common, ig, io = np.intersect1d(gk, ok, assume_unique=True, return_indices=True)
    # a pair on one side only is allowed only at the cut-off radius (binary32 test)
    a = orc.derived()["a"]
    for src, keys in ((gp, gk), (op, ok)):
        extra = ~np.isin(keys, common)
        r = src["R"][extra] * a
        near = np.abs(r - rcut) <= 1e-6 * rcut
        rep.pair_set_near_cut += int(near.sum())
        rep.pair_set_mismatch += int((~near).sum())
    g, o = gp[ig], op[io]
    decisions_ok = True
    if len(g):
        rep.max_dp = max(rep.max_dp, float(np.abs(g["p"] - o["p"]).max()))
        rep.draw_mismatch += int((g["draw"] != o["draw"]).sum())
        bad = g["cand"] != o["cand"]
        if bad.any():
            near = _near(o["draw"][bad], o["p"][bad], p_tol)
            rep.near_decisions += int(near.sum())
            rep.unexplained += int((~near).sum())
            decisions_ok = False
    # 4. picks
    gk2 = np.sort(_key(gpu.dbg_picks()["i"], gpu.dbg_picks()["j"]))
    pk = orc.picks()
    ok2 = np.sort(_key(pk["i"], pk["j"]))
    if decisions_ok and not np.array_equal(gk2, ok2):
        rep.notes.append(f"step {rep.steps}: picks differ")
        rep.unexplained += 1
        decisions_ok = False
    # 5. matches
    gmt, omt = gpu.dbg_matches(), orc.matches()
    rep.matches += len(omt)
    rep.reactions += int(omt["reacted"].sum())
    if decisions_ok:
        gs, os_ = gmt[np.argsort(_key(gmt["i"], gmt["j"]))], omt[np.argsort(_key(omt["i"], omt["j"]))]
        if len(gs) != len(os_) or not (np.array_equal(gs["i"], os_["i"]) and np.array_equal(gs["j"], os_["j"])):
            rep.notes.append(f"step {rep.steps}: matches differ")
            rep.unexplained += 1
            decisions_ok = False
        elif len(gs):
            rep.max_dRpp = max(rep.max_dRpp, float(np.abs(gs["Rpp"] - os_["Rpp"]).max()))
            rep.max_dpreac = max(rep.max_dpreac, float(np.abs(gs["preac"] - os_["preac"]).max()))
            rep.draw_mismatch += int((gs["draw"] != os_["draw"]).sum())
            # the angle of each propagated pair (NaN where none was drawn, on both sides)
            same = gs["reacted"] == os_["reacted"]
            gn, on = np.isnan(gs["cos_theta"][same]), np.isnan(os_["cos_theta"][same])
            if not np.array_equal(gn, on):
                rep.notes.append(f"step {rep.steps}: angles drawn for different pairs")
                rep.unexplained += 1
            elif (~on).any():
                d = np.abs(gs["cos_theta"][same][~on] - os_["cos_theta"][same][~on])
                rep.max_dcos = max(rep.max_dcos, float(d.max()))
                rep.angles += int((~on).sum())
            # a reaction flag may differ only where the draw lies within the tolerance of p_reac
            badr = gs["reacted"] != os_["reacted"]
            if badr.any():
                near = _near(os_["draw"][badr], os_["preac"][badr], p_tol)
                rep.near_decisions += int(near.sum())
                rep.unexplained += int((~near).sum())
                if (~near).any():
                    rep.notes.append(f"step {rep.steps}: reaction flags differ away from p_reac")
                decisions_ok = False
    # 6. dissociations
    gd, od = gpu.dbg_diss(), orc.dissociations()
    rep.decays += len(od)
    if decisions_ok:
        gs, os_ = gd[np.argsort(gd["c"])], od[np.argsort(od["c"])]
        if not np.array_equal(gs["c"], os_["c"]):
            rep.notes.append(f"step {rep.steps}: dissociations differ")
            rep.unexplained += 1
            decisions_ok = False
        elif len(gs):
            rep.max_dRpp = max(rep.max_dRpp, float(np.abs(gs["Rpp"] - os_["Rpp"]).max()))
            rep.draw_mismatch += int((gs["draw"] != os_["draw"]).sum())
            badg = gs["recombined"] != os_["recombined"]
            if badg.any():
                near = _near(os_["draw"][badg], os_["preac"][badg], p_tol)
                rep.near_decisions += int(near.sum())
                rep.unexplained += int((~near).sum())
                if (~near).any():
                    rep.notes.append(f"step {rep.steps}: geminate flags differ away from p_reac")
                decisions_ok = False
    # 7. state
    gsp, gpos, gpt = gpu.state()
    osp, opos, opt = orc.state()
    same = np.array_equal(gsp, osp)
    drift = False
    if same:
        lv = osp <= O.SP_C
        if lv.any():
            d = np.abs(gpos[lv] - opos[lv])
            d = np.minimum(d, box - d)
            rep.max_dpos = max(rep.max_dpos, float(d.max()))
            same = float(d.max()) <= pos_tol
            drift = float(d.max()) > 0.0
        cs = osp == O.SP_C
        same = same and np.array_equal(gpt[cs], opt[cs])
    if same and drift and lockstep:
        rep.pos_resyncs += 1
        gpu.load_state(orc.stepno, osp, opos, opt)
    if not same:
        if decisions_ok:
            rep.notes.append(f"step {rep.steps}: state differs without a decision difference")
            rep.unexplained += 1
        rep.resyncs += 1
        gpu.load_state(orc.stepno, osp, opos, opt)
    return osp


class MemberView:
    """One member of a batch or pool handle, seen by compare_step in the member's own slot
    numbering (slots lo .. lo + n - 1 of the handle become 0 .. n - 1).  Stepping it steps the
    whole handle.  Its logs are the handle's logs restricted to the member's slots; a member's
    pairs, picks, matches and dissociations never involve another member's slots.  There is no
    per-member reload, so a comparison that would need one fails."""

    def __init__(self, h, lo, n):
        self.h, self.lo, self.n = h, int(lo), int(n)

    def step(self):
        self.h.step()

    def _cut(self, log, key, shift):
        keep = (log[key] >= self.lo) & (log[key] < self.lo + self.n)
        out = log[keep].copy()
        for f in shift:
            if f in out.dtype.names:
                ok = out[f] != np.uint32(0xFFFFFFFF)
                out[f][ok] -= np.uint32(self.lo)
        return out

    def dbg_moved(self):
        return self.h.dbg_moved()[self.lo:self.lo + self.n]

    def dbg_pairs(self):
        full = self.h.dbg_pairs()
        if len(full) != self.h.stats()["pairs"]:
            raise AssertionError(f"GPU pair log truncated: {len(full)} of {self.h.stats()['pairs']} (raise debug_cap)")
        return self._cut(full, "i", ("i", "j"))

    def stats(self):
        return {"pairs": len(self.dbg_pairs())}

    def dbg_picks(self):
        return self._cut(self.h.dbg_picks(), "i", ("i", "j"))

    def dbg_matches(self):
        return self._cut(self.h.dbg_matches(), "i", ("i", "j"))

    def dbg_diss(self):
        return self._cut(self.h.dbg_diss(), "c", ("c", "j"))

    def state(self):
        sp, pos, pt = self.h.state()
        sl = slice(self.lo, self.lo + self.n)
        sp, pos, pt = sp[sl].copy(), pos[sl].copy(), pt[sl].copy()
        c = sp == S.SP_C
        pt[c] -= np.uint32(self.lo)
        return sp, pos, pt

    def load_state(self, *args, **kw):
        raise AssertionError("the member left the oracle's trajectory (a batch member cannot be reloaded alone)")


def run(gpu, orc, steps, *, p_tol, pos_tol, box, lockstep=None, stage=False):
    """lockstep: reload the GPU with the oracle's state after a step whose positions agree
    within pos_tol but not bit for bit.  By default on wherever angles are drawn: the two
    sides' roots of the angular distribution function differ in their last bits, which moves
    binary64 positions by about 1e-14 and the next step's p_enc by about 1e-12."""
    if lockstep is None:
        lockstep = not orc.keep_direction
    rep = Report()
    rcut = orc.derived()["rcut"]
    sp, _, _ = orc.state()
    for k in range(steps):
        sp = compare_step(gpu, orc, rep, p_tol=p_tol, pos_tol=pos_tol, box=box, rcut=rcut, sp_before=sp,
                          lockstep=lockstep, stage=stage)
        print(f"  step {k}: pairs {rep.pairs} matches {rep.matches} reactions {rep.reactions} "
              f"max|dp| {rep.max_dp:.2e} resyncs {rep.resyncs}", flush=True)
    return rep
