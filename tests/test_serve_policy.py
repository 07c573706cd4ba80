"""Admission policy of the serving loop, on the CPU with a stand-in pool: the HBM ledger is never
exceeded, a request that does not fit lets at most `max_bypass` later requests go ahead of it
(and is then admitted before anything else of its dimension), arrival order is kept when
nothing is bypassed, and every request completes.  The GPU pool itself is tested in
test_gpu_pool.py and test_gpu_serve.py."""
import numpy as np

from paper_1107_0270_amd import serve as V


class FakePool:
    """Slots as one counter (no fragmentation); admission, steps and retirement on the host."""

    def __init__(self, cap, log):
        self.cap, self.used, self.log, self.next = cap, 0, log, 0
        self.members = {}

    def try_admit(self, species, pos, box, replica=0):
        n = len(species)
        if self.used + n > self.cap:
            return None
        self.used += n
        self.next += 1
        self.members[self.next] = n
        self.log.append(("admit", replica))
        return self.next

    def step(self, k):
        pass

    def retire(self, m):
        self.used -= self.members.pop(m)

    def close(self):
        pass


def _trace(sizes, dims, steps):
    reqs = []
    for i, (n, d, s) in enumerate(zip(sizes, dims, steps)):
        r = V.Request(id=i, dim=d, n=n, steps=s, arrival=0.001 * i)
        r.species = np.zeros(n, np.int32)
        r.pos = np.zeros((n, d))
        r.box = 1.0
        reqs.append(r)
    return reqs


class CheckedServer(V.Server):
    def _take(self, fp):
        ok = super()._take(fp)
        assert self.ledger <= self.hbm_budget
        return ok


def _serve(reqs, cap, budget, max_bypass):
    log = []
    srv = CheckedServer(slot_cap={3: cap, 2: cap}, tick=7, read_results=False, hbm_budget=budget,
                        max_bypass=max_bypass, pool_factory=lambda d: FakePool(cap, log))
    srv.run(reqs, realtime=False)
    return srv, log


def test_ledger_bounds_both_pools_together():
    rng = np.random.default_rng(1)
    n = 200
    reqs = _trace(rng.integers(100, 3000, n), rng.choice([2, 3], n), rng.integers(5, 60, n))
    budget = 5000 * V.BYTES_PER_SLOT  # less than the two pools' 2 x 8000 slots
    srv, log = _serve(reqs, 8000, budget, 8)
    assert all(r.finished is not None for r in reqs)
    assert srv.ledger == 0 and 0 < srv.ledger_peak <= budget
    assert srv.ledger_peak > budget // 2  # the ledger, not the pools, was the bound


def test_head_of_line_is_bypassed_a_bounded_number_of_times():
    # one large request behind a running one of its size: small requests that arrive after it
    # may go first, at most max_bypass of them while it waits
    sizes = [6000, 7000] + [200] * 40
    reqs = _trace(sizes, [3] * len(sizes), [50, 10] + [3] * 40)
    for k in (0, 3, 8):
        for r in reqs:
            r.admitted = r.finished = None
            r.bypassed = 0
        srv, log = _serve(reqs, 8000, 10 ** 12, k)
        order = [rid for what, rid in log if what == "admit"]
        assert sorted(order) == list(range(len(sizes)))
        assert reqs[1].bypassed == min(k, 40)
        # requests admitted before the large one are exactly its bypassers
        assert order.index(1) == 1 + min(k, 40)
        if k == 0:
            assert order == sorted(order)  # plain arrival order


def test_request_larger_than_the_ledger_is_refused():
    reqs = _trace([3000], [3], [5])
    srv = V.Server(slot_cap={3: 8000, 2: 8000}, hbm_budget=1000 * V.BYTES_PER_SLOT, read_results=False,
                   pool_factory=lambda d: FakePool(8000, []))
    try:
        srv.run(reqs, realtime=False)
    except ValueError as e:
        assert "ledger" in str(e)
    else:
        raise AssertionError("not refused")
