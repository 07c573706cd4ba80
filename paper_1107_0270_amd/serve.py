"""Serving loop: continuous batching of simulation requests on one GPU.

Requests (a 2D or 3D system of N particles to run for S steps) arrive over time.  Each
dimension has a worker thread that owns one pool (sim_pool_create) on its own stream, so 2D
and 3D work proceeds on the device at the same time.  A worker repeatedly

  1. admits arrived requests of its dimension: a request is admitted when the server's HBM
     ledger (device bytes of all running requests, both pools, against one budget) has room
     for its footprint and its pool has a free range of slots and cells (sim_pool_admit).
     Requests go in arrival order, except that when the oldest waiting request does not fit,
     later arrived requests that fit may go ahead of it, at most `max_bypass` times for that
     request; after that nothing more is admitted in its dimension until it fits, so no
     request waits for ever;
  2. steps the pool up to the next completion (at most `tick` steps), and
  3. reads each finished request's final state and retires it, which frees its slots and
     returns its footprint to the ledger.

A request's result is the one it gets alone: the same draws (keyed on its replica number =
request id, its own slots and its own steps) and the same arithmetic, whoever shares the pool.
"""
from __future__ import annotations

import dataclasses
import threading
import time

import numpy as np

from . import inputs as I
from . import sim as S

# Device bytes a pool holds per slot (binary32 state): 112 B of records and slot arrays, 176 B of
# pair lists (4 pairs per slot), 18 B of bucket arrays (half a cell per slot).
BYTES_PER_SLOT = 306


@dataclasses.dataclass
class Request:
    id: int
    dim: int
    n: int
    steps: int
    arrival: float                     # seconds after the start of the run
    species: np.ndarray = None
    pos: np.ndarray = None
    box: float = 0.0
    # filled by the server
    admitted: float = None
    finished: float = None
    result: tuple = None               # (species, positions, partner) when kept
    bypassed: int = 0                  # later requests admitted ahead of this one


# Shared parameters of each dimension (3D: the radiation workload; 2D: the membrane workload at
# dt = 5 us), with the pair cut-off at a reaction probability of 1e-6 per step.  Per request: N,
# the box at the workload's density, the steps and the key.
GROUP_PARAMS = {
    3: dict(dim=3, dt=1e-5, D=(1.0, 1.0, 0.5), sigma=0.005, bc=S.BC_RADIATION, kappa=0.1, k_off=10.0, seed=0,
            precision=S.PREC_FP32D_FP64NC, eps_cut=1e-6),
    2: dict(dim=2, dt=5e-6, D=(0.1, 0.1, 0.05), sigma=0.005, bc=S.BC_RADIATION, kappa=0.05, k_off=10.0, seed=0,
            precision=S.PREC_FP32_FP64NC, eps_cut=1e-6),
}
DENSITY = {3: 1000.0, 2: 2500.0}  # particles per um^3 / um^2


def request_box(dim, n):
    return float(np.float32((n / DENSITY[dim]) ** (1.0 / dim)))


def make_trace(count, rate, seed=0, n_range=(1e3, 1e6), step_range=(100, 10_000), p3=0.5):
    """Poisson arrivals at `rate` per second; dimension 3 with probability p3; N and steps
    log-uniform in the given ranges; all draws from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    dims = np.where(rng.random(count) < p3, 3, 2)
    ns = np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]), count)).astype(np.int64)
    steps = np.exp(rng.uniform(np.log(step_range[0]), np.log(step_range[1]), count)).astype(np.int64)
    return [Request(id=i, dim=int(dims[i]), n=int(ns[i]), steps=int(steps[i]), arrival=float(t[i])) for i in range(count)]


def initial_state(req, redraw=True):
    """Uniform A and B (half each) at the workload density, binary32-exact, from PCG64(10000 + id),
    every B closer than sigma to an A redrawn.  `redraw=False` leaves overlapping pairs as drawn
    (at these densities about 3 in 10^4 B's start within sigma of an A; the step treats them as
    overlaps), which generates a large trace several times faster."""
    req.box = request_box(req.dim, req.n)
    n_a = req.n // 2
    if redraw:
        sp, pos, _ = I.uniform_state(n_a, req.n - n_a, box=req.box, dim=req.dim, sigma=0.005, seed=10_000 + req.id,
                                     f32=True)
    else:
        rng = np.random.Generator(np.random.PCG64(10_000 + req.id))
        pos = rng.random((req.n, req.dim), dtype=np.float32).astype(np.float64) * np.float32(req.box)
        pos = pos.astype(np.float32).astype(np.float64)
        pos[pos >= req.box] = 0.0
        sp = np.concatenate([np.full(n_a, S.SP_A, np.int32), np.full(req.n - n_a, S.SP_B, np.int32)])
    req.species, req.pos = sp, pos
    return req


def run_alone(req, keep=True):
    """The request on a handle of its own (the reference for 'the same alone and in the mix')."""
    p = dict(GROUP_PARAMS[req.dim])
    dim = p.pop("dim")
    sim = S.Sim(dim=dim, box=req.box, species=req.species, pos=req.pos, replica=req.id, **p)
    sim.step(req.steps)
    out = sim.state()
    sim.close()
    return out


def footprint(req):
    """Device bytes a request holds in its pool while it runs (the ledger's unit)."""
    return int(req.n) * BYTES_PER_SLOT


class _Running:
    def __init__(self, req):
        self.req = req
        self.done = 0  # steps taken


class Server:
    """Continuous-batching server: one pool per dimension with room for `slot_cap[dim]` slots
    (its cells: half as many, which covers about one cell per B) and `rep_cap` members."""

    def __init__(self, slot_cap=None, rep_cap=4096, tick=200, keep_results=False, read_results=None, progress=None,
                 hbm_budget=None, max_bypass=8, max_scan=64, pool_factory=None):
        self.slot_cap = dict(slot_cap or {3: 1 << 24, 2: 1 << 24})
        # the ledger: device bytes of running requests, both pools together (default: what the
        # two pools hold, so only the pools bound admission)
        self.hbm_budget = int(hbm_budget) if hbm_budget is not None else sum(self.slot_cap.values()) * BYTES_PER_SLOT
        self.ledger = 0
        self.ledger_peak = 0
        self.max_bypass = int(max_bypass)
        self.max_scan = int(max_scan)  # waiting requests looked at per admission round
        self.bypasses = 0
        self.pool_factory = pool_factory or self._pool
        self.read = keep_results if read_results is None else read_results  # read each final state
        self.progress = progress  # called with a line after every 100th completed request
        self.completed = 0
        self.rep_cap = rep_cap
        self.tick = tick
        self.keep = keep_results
        self.lock = threading.Lock()
        self.admissions = 0
        self.step_calls = 0
        self.admit_s = 0.0
        self.step_s = 0.0

    def run(self, requests, realtime=True):
        """Serve `requests` (with initial states) in arrival order; returns them completed."""
        for r in requests:
            if r.n > self.slot_cap[r.dim]:
                raise ValueError(f"request {r.id} needs {r.n} slots, the {r.dim}D pool has {self.slot_cap[r.dim]}")
            if footprint(r) > self.hbm_budget:
                raise ValueError(f"request {r.id} needs {footprint(r)} B of the {self.hbm_budget} B ledger")
        self.realtime = realtime
        ordered = sorted(requests, key=lambda r: r.arrival)
        self.pending = {d: [r for r in ordered if r.dim == d] for d in (2, 3)}
        self.errors = []
        # pools are created before the clock starts
        self.pools = {d: self.pool_factory(d) for d in (2, 3) if self.pending[d]}
        workers = [threading.Thread(target=self._worker, args=(d,)) for d in self.pools]
        self.t0 = time.perf_counter()
        for w in workers:
            w.start()
        for w in workers:
            w.join()
        self.t_end = time.perf_counter() - self.t0
        for p in self.pools.values():
            p.close()
        if self.errors:
            raise self.errors[0]
        return requests

    def now(self):
        return time.perf_counter() - self.t0

    def _pool(self, dim):
        p = dict(GROUP_PARAMS[dim])
        p.pop("dim")
        cap = self.slot_cap[dim]
        return S.Pool(dim=dim, box=request_box(dim, 1000), slot_cap=cap, cell_cap=cap // 2 + 4096,
                      rep_cap=self.rep_cap, **p)

    def _count(self, attr, dt, n=1):
        with self.lock:
            setattr(self, attr, getattr(self, attr) + dt)
            if attr == "admit_s":
                self.admissions += n
            else:
                self.step_calls += n

    def _take(self, fp):
        with self.lock:
            if self.ledger + fp > self.hbm_budget:
                return False
            self.ledger += fp
            self.ledger_peak = max(self.ledger_peak, self.ledger)
            return True

    def _give(self, fp):
        with self.lock:
            self.ledger -= fp

    def _admit_ready(self, pool, q, running):
        """Admit arrived requests of one dimension (see the module text); returns how many."""
        admitted, i = 0, 0
        while i < min(len(q), self.max_scan):
            r = q[i]
            if self.realtime and r.arrival > self.now():
                break  # not arrived yet (q is in arrival order)
            if i > 0 and q[0].bypassed >= self.max_bypass:
                break  # the oldest request has been passed over enough: it goes next
            fp = footprint(r)
            took = self._take(fp)
            m = pool.try_admit(r.species, r.pos, r.box, replica=r.id) if took else None
            if m is None:
                if took:
                    self._give(fp)  # the ledger had room, the pool had no free range
                i += 1  # no room for this one: a later arrived request may fit
                continue
            q.pop(i)
            if i > 0:
                q[0].bypassed += 1
                with self.lock:
                    self.bypasses += 1
            r.admitted = self.now()
            running[m] = _Running(r)
            admitted += 1
        return admitted

    def _worker(self, dim):
        try:
            pool, q = self.pools[dim], self.pending[dim]
            running = {}  # member entry -> _Running
            while running or q:
                t = time.perf_counter()
                admitted = self._admit_ready(pool, q, running)
                if admitted:
                    self._count("admit_s", time.perf_counter() - t, admitted)
                if not running:
                    if q:  # nothing arrived yet, or no room while the other pool holds the ledger
                        time.sleep(min(0.02, max(0.001, q[0].arrival - self.now())) if self.realtime else 0.001)
                    continue
                k = min(self.tick, min(x.req.steps - x.done for x in running.values()))
                t = time.perf_counter()
                pool.step(k)
                self._count("step_s", time.perf_counter() - t)
                for x in running.values():
                    x.done += k
                for m in [m for m, x in running.items() if x.done >= x.req.steps]:
                    x = running.pop(m)
                    if self.read:
                        out = pool.member_state(m)
                        if self.keep:
                            x.req.result = out
                    pool.retire(m)
                    self._give(footprint(x.req))
                    x.req.finished = self.now()
                    with self.lock:
                        self.completed += 1
                        done = self.completed
                    if self.progress and done % 100 == 0:
                        self.progress(f"[serve] {done} requests done at t = {x.req.finished:.1f} s, "
                                      f"{len(running)} running in the {dim}D pool, {len(q)} waiting")
        except Exception as e:  # surfaced by run()
            self.errors.append(e)

    def summary(self, requests):
        lat = np.array([r.finished - r.arrival for r in requests])
        work = sum(r.n * r.steps for r in requests)
        return {
            "requests": len(requests),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_queue_s": float(np.mean([r.admitted - r.arrival for r in requests])),
            "particle_steps": int(work),
            "wall_s": self.t_end,
            "particle_steps_per_s": work / self.t_end,
            "admissions": self.admissions,
            "bypasses": self.bypasses,
            "hbm_budget_bytes": self.hbm_budget,
            "ledger_peak_bytes": self.ledger_peak,
            "admit_s": self.admit_s,
            "step_calls": self.step_calls,
            "step_s": self.step_s,
        }
