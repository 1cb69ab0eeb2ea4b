"""Pins of the Cholesky-inversion oracle (oracle/cholinv.py) and of its task
graph (oracle/schedule.py, cholinv_dag) against what the thesis prints and
what the mathematics fixes:

* exact rational inverses of small integer SPD matrices (Gauss-Jordan in
  fractions), the closed-form inverse of the tridiagonal (-1, 2, -1)
  matrix, diagonal matrices, L L^T = A, W L = I;
* table table:criticalpath (chapter "Cholesky Inversion", section
  "Algorithmic study"): the critical path of each step in place and out of
  place with loop orders UDU, and the step-2 critical paths with UUU
  (t^2 - 2t + 3 in place, t^2/2 - t/2 + 2 out of place);
* task counts of the three steps and the weighted critical path 9t - 10 of
  step 1 (chapter "Scheduling of Cholesky Factorization")."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import cholinv as C
from oracle import schedule as S

EPS = np.finfo(np.float64).eps


def _exact_inverse(M):
    n = len(M)
    a = [[Fraction(int(M[i][j])) for j in range(n)] + [Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if a[r][c] != 0)
        a[c], a[p] = a[p], a[c]
        piv = a[c][c]
        a[c] = [v / piv for v in a[c]]
        for r in range(n):
            if r != c and a[r][c] != 0:
                f = a[r][c]
                a[r] = [x - f * y for x, y in zip(a[r], a[c])]
    return np.array([[float(v) for v in row[n:]] for row in a])


def test_exact_rational_inverses():
    rng = np.random.default_rng(11)
    for n in (1, 2, 3, 5, 8):
        for _ in range(3):
            M = rng.integers(-3, 4, size=(n, n))
            A = M.T @ M + np.eye(n, dtype=np.int64)
            X = C.spd_inverse(A.astype(np.float64))
            Xe = _exact_inverse(A)
            kap = np.linalg.cond(A)
            assert np.linalg.norm(X - Xe) <= 20 * n * kap * EPS * np.linalg.norm(Xe), n


def test_tridiagonal_closed_form():
    """(T^{-1})_{ij} = min(i,j) (n + 1 - max(i,j)) / (n + 1), 1-based, for
    T = tridiag(-1, 2, -1)."""
    for n in (1, 4, 17, 64):
        T = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
        i = np.arange(1, n + 1)
        ref = np.minimum.outer(i, i) * (n + 1 - np.maximum.outer(i, i)) / (n + 1)
        X = C.spd_inverse(T)
        assert np.allclose(X, ref, rtol=0, atol=8 * n * n * EPS * np.abs(ref).max())


def test_factor_and_triangular_inverse_definitions():
    rng = np.random.default_rng(3)
    G = rng.standard_normal((40, 40))
    A = G @ G.T + 40 * np.eye(40)
    L = C.cholesky(A)
    assert np.allclose(np.triu(L, 1), 0)
    assert np.all(np.diag(L) > 0)
    assert np.linalg.norm(L @ L.T - A) <= 40 * EPS * np.linalg.norm(A)
    W = C.lower_inverse(L)
    assert np.allclose(np.triu(W, 1), 0)
    assert np.linalg.norm(W @ L - np.eye(40)) <= 100 * EPS * np.linalg.cond(L)
    d = rng.uniform(0.5, 4.0, 9)
    assert np.allclose(C.spd_inverse(np.diag(d)), np.diag(1 / d), rtol=4 * EPS, atol=0)
    with pytest.raises(np.linalg.LinAlgError):
        C.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))


def test_planted_mistake_is_caught():
    """W W^T in place of W^T W (the transposition of step 3) is the inverse
    of L^T L, not of A: the tridiagonal pin rejects it."""
    n = 6
    T = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    W = C.lower_inverse(C.cholesky(T))
    i = np.arange(1, n + 1)
    ref = np.minimum.outer(i, i) * (n + 1 - np.maximum.outer(i, i)) / (n + 1)
    assert not np.allclose(W @ W.T, ref, atol=1e-6)


def _poly(s, t):
    a, b, c = (float(x) for x in s.split(","))
    return a * t * t + b * t + c


def test_table_criticalpath(golden):
    rows = {r[0]: r[1:] for r in golden("table_criticalpath.txt")}
    for t in range(2, 11):  # the closed forms are stated for t >= 2
        for inplace, col in ((True, 0), (False, 1)):
            steps = S.cholinv_step_cps(t, inplace, "UDU")
            for s in range(3):
                assert steps[s] == _poly(rows[str(s + 1)][col], t), (t, inplace, s)
            # steps separated: the critical paths add up
            assert S.critical_path(S.cholinv_dag(t, inplace, "UDU", pipelined=False)) == sum(steps)
            uuu = S.cholinv_step_cps(t, inplace, "UUU")
            assert uuu[1] == _poly(rows["UUU2"][col], t), (t, inplace)
            assert uuu[0] == steps[0] and uuu[2] == steps[2]


def test_cholinv_task_counts_and_weights():
    for t in range(1, 9):
        d = S.cholinv_dag(t, weights=S.CHOLINV_WEIGHTS)
        kinds = {}
        for nm in d.names:
            kinds[nm[0]] = kinds.get(nm[0], 0) + 1
        t2, t3 = t * (t - 1) // 2, t * (t - 1) * (t - 2) // 6
        assert kinds.get("POTRF", 0) == kinds.get("TRTRI", 0) == kinds.get("LAUUM", 0) == t
        assert kinds.get("TRSM", 0) == t2 and kinds.get("TRMM", 0) == 3 * t2
        assert kinds.get("SYRK", 0) == 2 * t2 and kinds.get("GEMM", 0) == 3 * t3
        # n^3 flops in all (n^3/3 per step) = 3 t^3 units of nb^3/3
        assert d.total_work() == 3 * t ** 3
        # step 1 alone is the tile Cholesky factorization: weighted cp 9t - 10
        d1 = S.cholesky_dag(t)
        assert S.critical_path(d1) == max(9 * t - 10, 1)
