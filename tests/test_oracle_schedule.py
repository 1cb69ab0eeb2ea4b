"""Pins of the bounded-resource scheduling oracle (oracle/schedule.py)
against what the thesis prints and what scheduling theory fixes:

* the weighted critical path 9t - 10 of the tile Cholesky factorization
  (chapter "Scheduling of Cholesky Factorization", introduction);
* figure fig:ALAP5x5 (the (processors, idle time) pairs) and table
  tab:bound5x5 (ALAP derived bound, speedup, efficiency), Cholesky 5 x 5;
* table tab:5x5_optimal (QR, 5 x 5 tiles): the ALAP derived bound of GrASAP
  on 1..14 processors and the CP-method schedules of GrASAP, Greedy,
  Fibonacci and FlatTree;
* the explicit QR task graph against the table-pinned tiled simulator
  (critical paths, zero times, kernel counts) for every tree and both
  kernel families;
* the two-processor example of section "Critical Path Scheduling" where the
  critical-path schedule is not optimal;
* invariants: every list schedule lies between the ALAP derived bound and
  Graham's bound T_seq / P + (1 - 1/P) cp."""
import math
import random

import pytest

from oracle import schedule as S
from oracle import trees as T


def test_cholesky_critical_path_closed_form():
    for t in range(1, 13):
        d = S.cholesky_dag(t)
        assert S.critical_path(d) == max(9 * t - 10, 1), t
        # t POTRF, t(t-1)/2 TRSM and SYRK, t(t-1)(t-2)/6 GEMM: t^3 units of nb^3/3
        assert d.total_work() == t ** 3


def test_fig_alap5x5_lost_area(golden):
    d = S.cholesky_dag(5)
    for p, la in golden("fig_alap5x5.txt"):
        assert S.lost_area(d, int(p)) == int(la), p


def test_tab_bound5x5(golden):
    d = S.cholesky_dag(5)
    assert d.total_work() == 125
    for p, tp, sp, ep in golden("tab_bound5x5.txt"):
        p = int(p)
        b = S.alap_bound(d, p)
        assert round(float(b), 2) == float(tp), p
        assert round(125 / float(b), 2) == float(sp), p
        assert round(125 / float(b) / p, 2) == float(ep), p


def _qr5(tree):
    return S.qr_dag(5, 5, T.elimination_list(tree, 5, 5))


# Cells of tab:5x5_optimal that depend on the order among equal priorities
# (the thesis does not state its rule; the printed length is 2 above the
# one this tie rule gives), and the Fibonacci P = 14 entry, which is below
# Fibonacci's own unbounded critical path of 86 (a misprint).
TIE_CELLS = {("grasap", 3), ("grasap", 5), ("greedy", 3), ("greedy", 5), ("fibonacci", 3), ("fibonacci", 5)}
MISPRINT = {("fibonacci", 14)}


def test_tab_5x5_optimal(golden):
    rows = [[int(v) for v in r] for r in golden("tab_5x5_optimal.txt")]
    assert [r[0] for r in rows] == list(range(1, 15))
    dags = {t: _qr5(t) for t in ("grasap", "greedy", "fibonacci", "flat")}
    assert all(d.total_work() == 500 for d in dags.values())
    asserted = 0
    for r in rows:
        P = r[0]
        # ALAP derived bound of GrASAP; a schedule length is an integer, so
        # the printed bound is the ceiling of (T_seq + LA_P) / P
        assert math.ceil(S.alap_bound(dags["grasap"], P)) == r[1], P
        # the optimal tree/schedule lies between the bounds (IP not rebuilt)
        assert r[2] <= r[3]
        for col, tree in zip(r[3:], ("grasap", "greedy", "fibonacci", "flat")):
            got, _ = S.list_schedule(dags[tree], P)
            if (tree, P) in MISPRINT:
                assert got == S.critical_path(dags[tree]) == 86 > col
            elif (tree, P) in TIE_CELLS:
                assert got == col - 2
                assert got >= math.ceil(S.alap_bound(dags[tree], P))
            else:
                assert got == col, (tree, P)
                asserted += 1
    assert asserted == 14 * 4 - len(TIE_CELLS) - len(MISPRINT)


@pytest.mark.parametrize("mode", ["tt", "hybrid"])
def test_qr_dag_matches_the_tiled_simulator(mode):
    """The explicit graph's ASAP execution equals the tiled model that the
    printed tables pin: critical path, the time each tile is zeroed, and
    the kernel counts."""
    m = T.TT if mode == "tt" else T.HYBRID
    for (p, q) in [(4, 2), (8, 3), (15, 6), (5, 5), (20, 6), (7, 7)]:
        for tree in ("flat", "binary", "fibonacci", "greedy", "grasap", "asap"):
            el = T.elimination_list(tree, p, q)
            d = S.qr_dag(p, q, el, mode)
            ref = T.tiled(p, q, el, m)
            st = S.asap_times(d)
            assert S.critical_path(d) == ref["cp"], (tree, p, q)
            for t, name in enumerate(d.names):
                if name[0] in ("TTQRT", "TSQRT"):
                    i, k = name[1], name[3]
                    assert st[t] + d.w[t] == ref["zero"][i - 1, k - 1], (tree, p, q, name)
            counts = {}
            for name in d.names:
                counts[name[0]] = counts.get(name[0], 0) + 1
            for kname, c in ref["counts"].items():
                assert counts.get(kname, 0) == c, (tree, p, q, kname)


def test_critical_path_schedule_is_not_always_optimal():
    """Section "Critical Path Scheduling": two processors, A and B of weight
    3, C -> D of weight 1 each; the critical-path schedule takes 5, the
    optimum is 4."""
    d = S.Dag()
    d.add("A", 3, writes=["a"])
    d.add("B", 3, writes=["b"])
    d.add("C", 1, writes=["c"])
    d.add("D", 1, reads=["c"], writes=["d"])
    assert S.bottom_levels(d) == [3, 3, 2, 1]
    assert S.list_schedule(d, 2)[0] == 5
    assert S.alap_bound(d, 2) == 4


def _check_schedule(d, P, start):
    for t, pr in enumerate(d.preds):
        for u in pr:
            assert start[t] >= start[u] + d.w[u]
    ev = sorted([(start[t], 1) for t in range(len(d.w))] + [(start[t] + d.w[t], -1) for t in range(len(d.w))],
                key=lambda e: (e[0], e[1]))
    busy = 0
    for _, e in ev:
        busy += e
        assert busy <= P


def test_schedules_lie_between_the_bounds():
    rng = random.Random(5)
    for _ in range(12):
        p = rng.randint(2, 12)
        q = rng.randint(1, p)
        tree = rng.choice(["flat", "binary", "fibonacci", "greedy", "grasap"])
        mode = rng.choice(["tt", "hybrid"])
        d = S.qr_dag(p, q, T.elimination_list(tree, p, q), mode)
        cp, tseq = S.critical_path(d), d.total_work()
        for P in (1, 2, 3, 5, 8, 16, 64):
            lb = S.alap_bound(d, P)
            assert lb >= max(cp, tseq / P)
            for prio in (None, [rng.random() for _ in d.w]):
                mk, start = S.list_schedule(d, P, prio)
                _check_schedule(d, P, start)
                assert lb <= mk <= tseq / P + (1 - 1 / P) * cp + 1e-9, (tree, p, q, P)
    for t in range(2, 8):
        d = S.cholesky_dag(t)
        for P in (1, 2, 4, 7):
            mk, start = S.list_schedule(d, P)
            _check_schedule(d, P, start)
            assert S.alap_bound(d, P) <= mk


def test_planted_mistake_is_caught(golden):
    """A plausible mistake in the lost area (counting the whole execution
    instead of the tail that needs at most P processors) breaks the
    fig:ALAP5x5 pin."""
    d = S.cholesky_dag(5)
    prof = S.alap_profile(d)

    def wrong(P):
        return sum(max(P - x, 0) for x in prof)

    assert any(wrong(int(p)) != int(la) for p, la in golden("fig_alap5x5.txt"))
