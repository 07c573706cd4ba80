"""The serving loop: requests that arrive while others run join the running pool as slots free
up, and every request's result is exactly the one it gets alone."""
import numpy as np
import pytest

from paper_1107_0270_amd import serve as V
from paper_1107_0270_amd import sim as S

pytestmark = pytest.mark.gpu


def _check_alone(reqs):
    for r in reqs:
        sp1, pos1, pt1 = V.run_alone(r)
        sp, pos, pt = r.result
        assert np.array_equal(sp, sp1), r.id
        live = sp1 <= S.SP_C
        assert np.array_equal(pos[live], pos1[live]), r.id
        c = sp1 == S.SP_C
        assert np.array_equal(pt[c], pt1[c]), r.id


def test_each_result_is_the_same_alone_and_in_the_mix():
    rng = np.random.default_rng(4)
    reqs = []
    for i in range(10):
        dim = 3 if i % 2 == 0 else 2
        reqs.append(V.Request(id=i, dim=dim, n=int(rng.integers(800, 6000)), steps=int(rng.integers(20, 120)),
                              arrival=0.01 * i))
    for r in reqs:
        V.initial_state(r)
    srv = V.Server(slot_cap={3: 1 << 16, 2: 1 << 16}, tick=25, keep_results=True)
    srv.run(reqs)
    summ = srv.summary(reqs)
    print(summ)
    assert summ["admissions"] == len(reqs)
    _check_alone(reqs)


def test_requests_wait_for_slots_to_free_up():
    # a pool that holds one request at a time: they run one after another, results unchanged
    reqs = [V.Request(id=20 + i, dim=3, n=3000, steps=30, arrival=0.0) for i in range(3)]
    for r in reqs:
        V.initial_state(r)
    srv = V.Server(slot_cap={3: 4000, 2: 4000}, tick=10, keep_results=True)
    srv.run(reqs)
    assert reqs[1].admitted >= reqs[0].finished - 1e-3 and reqs[2].admitted >= reqs[1].finished - 1e-3
    _check_alone(reqs)


def test_trace_generator_is_seeded():
    a = V.make_trace(50, 200.0, seed=1)
    b = V.make_trace(50, 200.0, seed=1)
    assert [(r.dim, r.n, r.steps, r.arrival) for r in a] == [(r.dim, r.n, r.steps, r.arrival) for r in b]
