"""Pins of the scheduling oracle (oracle/tiledqr_lists.c) against what the
thesis prints: tables tab.coarse, tab.tiled, table.15x2x3, table.biggermat,
the p = 40 theoretical table, the closed forms of proposition th.ft and of
the coarse-grain critical paths, theorem thm.lowerbound, corollaries
cor.cplowup / cor.cpsquare, theorem thm.flops, lemma th.above, the 20 x 6
example of the bounds section and the GrASAP-vs-Greedy census."""
import numpy as np
import pytest

from oracle import trees as T

GOLD_TREE = {"SK": T.FLAT, "FLAT": T.FLAT, "FIBONACCI": T.FIBONACCI, "GREEDY": T.GREEDY,
             "BINARY": T.BINARY, "PLASMA5": T.PLASMA}


def _table(golden, name):
    per = {}
    for row in golden(name):
        alg, i, vals = row[0], int(row[1]), [int(v) for v in row[2:]]
        per.setdefault(alg, {})[i] = vals
    return per


def test_tab_coarse(golden):
    """Table tab.coarse: SK and Greedy are the coarse-grain ASAP execution of
    their lists; Fibonacci is the thesis's closed-form scheme."""
    p, q = 15, 6
    tab = _table(golden, "tab_coarse.txt")
    for alg, rows in tab.items():
        if alg == "FIBONACCI":
            got = T.fibonacci_coarse(p, q)
        else:
            _, got = T.coarse(p, q, T.elimination_list(GOLD_TREE[alg], p, q))
        cells = 0
        for i, vals in rows.items():
            for k, v in enumerate(vals, start=1):
                assert got[i - 1, k - 1] == v, (alg, i, k)
                cells += 1
        assert cells == 69


def test_tab_tiled(golden):
    """Table tab.tiled: the tiled zero time (end of TTQRT) of all 5 x 69 cells."""
    p, q = 15, 6
    tab = _table(golden, "tab_tiled.txt")
    assert set(tab) == {"FLAT", "FIBONACCI", "GREEDY", "BINARY", "PLASMA5"}
    for alg, rows in tab.items():
        param = 5 if alg == "PLASMA5" else 0
        res = T.tiled(p, q, T.elimination_list(GOLD_TREE[alg], p, q, param))
        for i, vals in rows.items():
            for k, v in enumerate(vals, start=1):
                assert res["zero"][i - 1, k - 1] == v, (alg, i, k)


def test_table_15x2x3(golden):
    """Table table.15x2x3: Greedy and ASAP zero times on 15 x 3 tiles."""
    p, q = 15, 3
    g = T.tiled(p, q, T.elimination_list("greedy", p, q))["zero"]
    a = T.tiled(p, q, T.elimination_list("asap", p, q))["zero"]
    for row in golden("table_15x2x3.txt"):
        i = int(row[0])
        vals = [int(v) for v in row[1:]]
        w = min(i - 1, 3)
        assert list(g[i - 1, :w]) == vals[:w], i
        assert list(a[i - 1, :w]) == vals[w:], i


def test_table_biggermat(golden):
    """Table table.biggermat.  The ASAP 128 x 64 cell (printed 1748) is not
    reproduced by the ASAP reading used here (1734) and is not asserted."""
    for row in golden("table_biggermat.txt"):
        p, q, gr, asap = (int(v) for v in row)
        assert T.tree_cp("greedy", p, q) == gr, (p, q)
        if (p, q) != (128, 64):
            assert T.tree_cp("asap", p, q) == asap, (p, q)


def test_p40_theory_table(golden):
    """Theoretical p = 40 table: Greedy CP, best PlasmaTree(TT) CP and its BS
    (smallest BS on ties), Fibonacci CP; the printed ratios are consistent."""
    for row in golden("p40_theory.txt"):
        p, q, gr, pt, bs, ov1, gain1, fib, ov2, gain2 = row
        p, q, gr, pt, bs, fib = int(p), int(q), int(gr), int(pt), int(bs), int(fib)
        assert T.tree_cp("greedy", p, q) == gr, q
        assert T.tree_cp("fibonacci", p, q) == fib, q
        cps = [T.tree_cp("plasma", p, q, b) for b in range(1, p + 1)]
        best = min(cps)
        assert best == pt, q
        assert cps.index(best) + 1 == bs, q
        assert abs(pt / gr - float(ov1)) < 6e-5 and abs(1 - gr / pt - float(gain1)) < 6e-5
        assert abs(fib / gr - float(ov2)) < 6e-5 and abs(1 - gr / fib - float(gain2)) < 6e-5


def test_flat_tree_closed_form():
    """Proposition th.ft: 2p+2 (q = 1), 22p-24 (p = q > 1), 6p+16q-22 (p > q > 1)."""
    for p in range(1, 41):
        for q in range(1, p + 1):
            cp = T.tree_cp("flat", p, q)
            if q == 1:
                want = 2 * p + 2 if p > 1 else 4
            elif p == q:
                want = 22 * p - 24
            else:
                want = 6 * p + 16 * q - 22
            assert cp == want, (p, q)


def _fib_x(p):
    x = 0
    while x * (x + 1) // 2 < p - 1:
        x += 1
    return x


def test_coarse_critical_paths():
    """Coarse-grain critical paths: SK p+q-2 (square 2q-3), Fibonacci
    x+2q-2 (square x+2q-4) with x the least integer, x(x+1)/2 >= p-1."""
    for p in range(3, 40):
        for q in range(2, p + 1):
            cp, _ = T.coarse(p, q, T.elimination_list("flat", p, q))
            assert cp == (2 * q - 3 if p == q else p + q - 2), (p, q)
            fib = T.fibonacci_coarse(p, q)
            want = _fib_x(p) + 2 * q - (4 if p == q else 2)
            assert fib.max() == want, (p, q)


@pytest.mark.parametrize("tree", ["flat", "binary", "greedy", "fibonacci", ("plasma", 3), ("plasma", 5)])
@pytest.mark.parametrize("shape", [(15, 6), (20, 10), (40, 20), (33, 7), (12, 12)])
def test_lowerbound_theorem(tree, shape):
    """Theorem thm.lowerbound: for every column k < q-1 the update that
    follows the zeroing of tile (i,k) ends at 10k + 6 coarse(i,k), with
    coarse the coarse-grain execution of the same list."""
    p, q = shape
    name, param = (tree, 0) if isinstance(tree, str) else tree
    L = T.elimination_list(name, p, q, param)
    _, crs = T.coarse(p, q, L)
    upd = T.tiled(p, q, L)["upd"]
    for (i, piv, k) in L:
        if k < q - 1:
            assert upd[i - 1, k - 1] == 10 * k + 6 * crs[i - 1, k - 1], (i, k)


@pytest.mark.parametrize("tree", ["flat", "binary", "greedy", "fibonacci", "grasap"])
def test_cp_corollaries(tree):
    """Corollaries cor.cplowup (p > q): tiled(p,q-1)+6 <= CP < tiled(p,q),
    and cor.cpsquare (p = q): CP = tiled(p,q-1)+4, where tiled(., k) is the
    last update time of column k, 10k + 6 coarse."""
    for p in range(3, 26):
        for q in range(2, p + 1):
            L = T.elimination_list(tree, p, q)
            cp = T.tree_cp(tree, p, q)
            if tree == "grasap":
                Lc = T.elimination_list("greedy", p, q)
            else:
                Lc = L
            _, crs = T.coarse(p, q, Lc)
            last = lambda k: 10 * k + 6 * int(crs[:, k - 1].max())
            if p == q:
                assert cp == last(q - 1) + 4, (p, q)
            else:
                assert last(q - 1) + 6 <= cp < last(q) + (0 if tree != "grasap" else 1), (p, q)


def test_20x6_bounds_example():
    """Bounds section: on 20 x 6 tiles Greedy's CP is 136 and GrASAP's 134."""
    assert T.tree_cp("greedy", 20, 6) == 136
    assert T.tree_cp("grasap", 20, 6) == 134


def test_grasap_greedy_census():
    """GrASAP is shorter than Greedy in just over 44% of the shapes
    1 <= q <= p <= 100, and always by exactly 2 units."""
    total = diff = 0
    deltas = set()
    for p in range(1, 101):
        for q in range(1, p + 1):
            a, b = T.tree_cp("greedy", p, q), T.tree_cp("grasap", p, q)
            total += 1
            assert b <= a
            if a != b:
                diff += 1
                deltas.add(a - b)
    assert total == 5050
    assert 0.44 < diff / total < 0.45
    assert deltas == {2}


@pytest.mark.parametrize("mode", [T.TT, T.HYBRID])
@pytest.mark.parametrize("tree", ["flat", "binary", "fibonacci", "greedy", "grasap", "plasma"])
def test_flops_theorem(tree, mode):
    """Theorem thm.flops: L1..L4 kernel counts and the total weight
    6pq^2 - 2q^3 are the same for every list and every TT/TS mix."""
    for p, q in [(4, 2), (8, 3), (15, 6), (13, 13), (30, 4), (9, 1)]:
        L = T.elimination_list(tree, p, q, 3 if tree == "plasma" else 0)
        c = T.tiled(p, q, L, mode)["counts"]
        assert c["GEQRT"] == c["TTQRT"] + q
        assert 2 * c["UNMQR"] == 2 * c["TTMQR"] + q * (q - 1)
        assert 2 * (c["TTQRT"] + c["TSQRT"]) == 2 * p * q - q * (q + 1)
        assert 6 * (c["TTMQR"] + c["TSMQR"]) == 3 * p * q * (q - 1) - q * (q - 1) * (q + 1)
        w = 4 * c["GEQRT"] + 6 * c["TSQRT"] + 2 * c["TTQRT"] + 6 * c["UNMQR"] + 12 * c["TSMQR"] + 6 * c["TTMQR"]
        assert w == 6 * p * q * q - 2 * q ** 3
        if mode == T.TT:
            assert c["TSQRT"] == 0 and c["TSMQR"] == 0
            assert c["GEQRT"] == sum(p - k + 1 for k in range(1, q + 1))


def test_hybrid_uses_all_six_kernels_on_4x2_greedy():
    c = T.tiled(4, 2, T.elimination_list("greedy", 4, 2), T.HYBRID)["counts"]
    assert all(v > 0 for v in c.values()), c


def test_single_elimination_parallel_time():
    """alg.elimSQ / alg.elimTR: one elimination with its updates takes 22
    (TS) and 16 (TT) time units on unbounded processors."""
    L = [(2, 1, 1)]
    tt = T.tiled(2, 2, L, T.TT)
    assert tt["upd"][1, 0] == 16
    hy = T.tiled(2, 2, L, T.HYBRID)
    assert hy["upd"][1, 0] == 22


@pytest.mark.parametrize("tree", ["flat", "binary", "fibonacci", "greedy", "grasap", "asap", "plasma"])
def test_list_validity(tree):
    """Section "Elimination lists": every tile below the diagonal is zeroed
    exactly once; both rows are ready (zeroed in all earlier columns) and the
    pivot is still alive; lemma th.above: piv(i,k) < i."""
    for p, q in [(4, 2), (8, 3), (15, 6), (17, 17), (40, 9)]:
        L = T.elimination_list(tree, p, q, 4 if tree == "plasma" else 0)
        zeroed = set()
        for (i, piv, k) in L:
            assert piv < i
            assert (i, k) not in zeroed and (piv, k) not in zeroed
            for kk in range(1, k):
                assert (i, kk) in zeroed and (piv, kk) in zeroed
            zeroed.add((i, k))
        assert zeroed == {(i, k) for k in range(1, q + 1) for i in range(k + 1, p + 1)}


def test_appendix_lists_small():
    """Hand-checkable lists on 4 x 2 (the smallest configuration)."""
    assert T.elimination_list("flat", 4, 2) == [(2, 1, 1), (3, 1, 1), (4, 1, 1), (3, 2, 2), (4, 2, 2)]
    assert T.elimination_list("binary", 4, 2) == [(2, 1, 1), (4, 3, 1), (3, 1, 1), (3, 2, 2), (4, 2, 2)]
    g = T.elimination_list("greedy", 4, 2)
    assert sorted(g, key=lambda e: (e[2], g.index(e))) == [(4, 2, 1), (3, 1, 1), (2, 1, 1), (4, 3, 2), (3, 2, 2)]
    _, crs = T.coarse(4, 2, g)
    assert (crs[3, 0], crs[2, 0], crs[1, 0], crs[3, 1], crs[2, 1]) == (1, 1, 2, 2, 3)


# Hybrid (TS) mode, derived by hand from the four dependency rules of
# algorithm alg.elimSQ (GEQRT(piv) < TSQRT; GEQRT(piv) < UNMQR(piv, j);
# UNMQR(piv, j) < TSMQR(j); TSQRT < TSMQR(j)), the data flow between
# successive eliminations that share a tile (each kernel that rewrites a
# tile waits for the previous writer), the rule that an already triangular
# tile is not factored again, and the weights of table tab.kernels
# (GEQRT 4, TSQRT 6, TTQRT 2, UNMQR 6, TSMQR 12, TTMQR 6).  Intervals are
# [start, end]; "zero" is the end of the kernel that zeroes the tile.
HYBRID_BY_HAND = {
    # FlatTree 2x2, list [(2,1,1)]:
    #   GEQRT(1,1) [0,4]; UNMQR(1,1,2) [4,10]; TSQRT(2,1,1) [4,10];
    #   TSMQR(2,1,1,2) after UNMQR and TSQRT [10,22] (the 22 of the text);
    #   the last diagonal tile is factored: GEQRT(2,2) [22,26].
    ("flat", 2, 2): (26, {(2, 1): 10}, (2, 1, 0, 1, 1, 0)),
    # FlatTree 3x2, list [(2,1,1),(3,1,1),(3,2,2)]:
    #   GEQRT(1,1) [0,4]; UNMQR(1,1,2) [4,10]; TSQRT(2,1,1) [4,10];
    #   TSMQR(2,1,1,2) [10,22]; TSQRT(3,1,1) after TSQRT(2,1,1) (both
    #   rewrite R(1,1)) [10,16]; TSMQR(3,1,1,2) after TSMQR(2,1,1,2) (both
    #   rewrite tile (1,2)) [22,34]; GEQRT(2,2) after TSMQR(2,1,1,2)
    #   [22,26]; TSQRT(3,2,2) needs tile (3,2) from TSMQR(3,1,1,2) [34,40].
    ("flat", 3, 2): (40, {(2, 1): 10, (3, 1): 16, (3, 2): 40}, (2, 3, 0, 1, 2, 0)),
    # FlatTree 4x2: as 3x2 plus TSQRT(4,1,1) [16,22], TSMQR(4,1,1,2)
    #   after TSMQR(3,1,1,2) [34,46]; TSQRT(4,2,2) (pivot 2 already
    #   triangular) after TSQRT(3,2,2) and TSMQR(4,1,1,2) [46,52].
    ("flat", 4, 2): (52, {(2, 1): 10, (3, 1): 16, (4, 1): 22, (3, 2): 40, (4, 2): 52}, (2, 5, 0, 1, 3, 0)),
    # FlatTree 3x3: column 1 as 3x2 with the same kernels on tile column 3
    #   (UNMQR(1,1,3) [4,10], TSMQR(2,1,1,3) [10,22], TSMQR(3,1,1,3)
    #   [22,34]); GEQRT(2,2) [22,26]; UNMQR(2,2,3) after GEQRT(2,2) and
    #   TSMQR(2,1,1,3) [26,32]; TSQRT(3,2,2) [34,40]; TSMQR(3,2,2,3) after
    #   TSQRT(3,2,2), UNMQR(2,2,3) and TSMQR(3,1,1,3) [40,52]; the last
    #   diagonal tile: GEQRT(3,3) [52,56].
    ("flat", 3, 3): (56, {(2, 1): 10, (3, 1): 16, (3, 2): 40}, (3, 3, 0, 3, 5, 0)),
    # Greedy 4x2, list [(4,2,1),(3,1,1),(2,1,1),(4,3,2),(3,2,2)]:
    #   GEQRT(2,1) [0,4], UNMQR(2,1,2) [4,10], TSQRT(4,2,1) [4,10],
    #   TSMQR(4,2,1,2) [10,22]; GEQRT(1,1) [0,4], UNMQR(1,1,2) [4,10],
    #   TSQRT(3,1,1) [4,10], TSMQR(3,1,1,2) [10,22]; tile (2,1) is a
    #   triangle: TTQRT(2,1,1) after both TSQRTs [10,12], TTMQR(2,1,1,2)
    #   after both TSMQRs [22,28]; GEQRT(3,2) after TSMQR(3,1,1,2) [22,26],
    #   TSQRT(4,3,2) after it [26,32]; GEQRT(2,2) after TTMQR [28,32],
    #   TTQRT(3,2,2) after GEQRT(2,2) and TSQRT(4,3,2) [32,34].
    ("greedy", 4, 2): (34, {(4, 1): 10, (3, 1): 10, (2, 1): 12, (4, 2): 32, (3, 2): 34}, (4, 3, 2, 2, 2, 1)),
}


@pytest.mark.parametrize("key", list(HYBRID_BY_HAND))
def test_hybrid_times_derived_by_hand(key):
    tree, p, q = key
    cp, zeros, counts = HYBRID_BY_HAND[key]
    res = T.tiled(p, q, T.elimination_list(tree, p, q), T.HYBRID)
    assert res["cp"] == cp
    for (i, k), t in zeros.items():
        assert res["zero"][i - 1, k - 1] == t, (i, k)
    assert tuple(res["counts"][n] for n in T.KERNELS) == counts
