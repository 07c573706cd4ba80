"""Autotuner host logic: candidate grids follow the library's grid rule, duplicates are
dropped, and the cache keeps choices per workload signature."""
import json

from paper_1107_0270_amd import autotune as AT
from paper_1107_0270_amd import sim as S


def test_grid_rule():
    # edge >= r_cut; fewer than three cells on an axis means one; at most 2048 per axis
    assert AT.grid_of(1.0, 3, 0.1, 0.02) == (10, 10, 10)
    assert AT.grid_of(1.0, 3, 0.01, 0.02) == (50, 50, 50)   # clamped to r_cut
    assert AT.grid_of(1.0, 2, 0.4, 0.02) == (1, 1)           # two cells per axis -> one
    assert AT.grid_of(100.0, 2, 0.01, 0.01) == (2048, 2048)
    assert AT.grid_of([2.0, 1.0, 1.0], 3, 0.25, 0.1) == (8, 4, 4)


def test_candidates_are_distinct_grids_with_each_search():
    c = AT.candidates(1.0, 3, 0.3, factors=(1.0, 1.05, 1.1), default_factors=())
    # 1.0 and 1.05 x 0.3 give the same 3x3x3 grid; 1.1 x 0.3 = 0.33 gives 3x3x3 too
    grids = {AT.grid_of(1.0, 3, cell, 0.3) for cell, _ in c if cell > 0}
    assert grids == {(3, 3, 3)}
    assert [ps for cell, ps in c if cell == 0.0] == list(AT.SEARCHES)
    assert len(c) == 2 * len(AT.SEARCHES)


def test_candidates_around_the_default_edge():
    # r_cut 0.02, default edge 0.1 on a unit box: multiples of both, none below r_cut, none
    # repeating the default grid (10^3) or each other
    c = AT.candidates(1.0, 3, 0.02, cell0=0.1, factors=(0.5, 1.0, 2.0), default_factors=(0.1, 0.95, 1.5))
    cells = sorted({cell for cell, _ in c})
    assert cells[0] == 0.0 and all(x >= 0.02 for x in cells[1:])
    grids = [AT.grid_of(1.0, 3, x, 0.02) for x in cells[1:]]
    assert len(grids) == len(set(grids)) and (10, 10, 10) not in grids
    assert (6, 6, 6) in grids and (50, 50, 50) in grids and (25, 25, 25) in grids


def test_signature_bins_and_cache_roundtrip(tmp_path):
    a = AT.signature(dim=3, precision=S.PREC_FP32_FP64NC, bc=S.BC_RADIATION, n=10**6, box=10.0, tau=0.8)
    b = AT.signature(dim=3, precision=S.PREC_FP32_FP64NC, bc=S.BC_RADIATION, n=10**6 + 1000, box=10.0, tau=0.81)
    c = AT.signature(dim=3, precision=S.PREC_FP32_FP64NC, bc=S.BC_RADIATION, n=10**6, box=5.0, tau=0.8)
    assert a == b and a != c
    path = str(tmp_path / "tune.json")
    cache = AT.TuneCache(path)
    cache.put(a, {"cell": 0.05, "pair_search": S.PAIRS_DIRECT})
    again = AT.TuneCache(path)
    assert again.get(a) == {"cell": 0.05, "pair_search": S.PAIRS_DIRECT}
    assert again.get(c) is None
    assert json.load(open(path))[a]["cell"] == 0.05
