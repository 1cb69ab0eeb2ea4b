"""Pins of the numeric oracle (oracle/householder.py) against the
mathematics: brute-force R from exact Gram matrices, exact special cases,
orthogonality, and exact rational least-squares solutions.  A planted
mistake in the oracle's reflector must be caught by these pins."""
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import householder as H

EPS = np.finfo(np.float64).eps


def _int_matrix(m, n, seed):
    rng = np.random.default_rng(seed)
    while True:
        A = rng.integers(-3, 4, size=(m, n)).astype(np.float64)
        if np.linalg.matrix_rank(A) == n:
            return np.asfortranarray(A)


def _chol_r_decimal(A, digits=50):
    """R with positive diagonal and R^T R = A^T A, from the exact integer
    Gram matrix by the Cholesky recurrence in 50-digit decimal arithmetic."""
    getcontext().prec = digits
    m, n = A.shape
    G = [[Decimal(int(sum(int(A[r, i]) * int(A[r, j]) for r in range(m)))) for j in range(n)] for i in range(n)]
    R = [[Decimal(0)] * n for _ in range(n)]
    for j in range(n):
        s = G[j][j] - sum(R[k][j] * R[k][j] for k in range(j))
        R[j][j] = s.sqrt()
        for c in range(j + 1, n):
            R[j][c] = (G[j][c] - sum(R[k][j] * R[k][c] for k in range(j))) / R[j][j]
    return np.array([[float(v) for v in row] for row in R])


@pytest.mark.parametrize("shape,seed", [((4, 2), 0), ((8, 3), 1), ((16, 8), 2), ((9, 9), 3), ((12, 5), 4)])
def test_r_matches_bruteforce_cholesky(shape, seed):
    A = _int_matrix(*shape, seed)
    R, V, tau = H.qr(A)
    Rref = _chol_r_decimal(A)
    Ra, _ = H.row_sign_align(R, Rref)
    kappa = np.linalg.cond(A)
    err = np.abs(Ra - Rref).max() / np.abs(Rref).max()
    assert err <= 20 * kappa * EPS, err
    assert np.allclose(np.tril(R, -1), 0.0)


def test_orthonormal_columns_give_unit_r():
    Q0 = synth.haar_orthogonal(50, 7)[:, :20]
    R, V, tau = H.qr(Q0)
    assert np.abs(np.abs(np.diag(R)) - 1).max() < 20 * EPS
    assert np.abs(np.triu(R, 1)).max() < 20 * EPS


def test_upper_triangular_input_is_its_own_r():
    rng = np.random.default_rng(3)
    A = np.triu(rng.standard_normal((30, 30)))
    A = np.vstack([A, np.zeros((10, 30))])
    R, V, tau = H.qr(A)
    assert np.array_equal(R, A[:30])
    assert np.array_equal(tau, np.zeros(30))


def test_power_of_two_scaling_is_exact():
    A = synth.gaussian(37, 19, 11)
    R1, _, _ = H.qr(A)
    R2, _, _ = H.qr(A * 2.0 ** 40)
    assert np.array_equal(R2, R1 * 2.0 ** 40)


@pytest.mark.parametrize("m,n", [(200, 80), (64, 64), (33, 1)])
def test_factorization_and_orthogonality(m, n):
    A = synth.gaussian(m, n, m + n)
    R, V, tau = H.qr(A)
    Q = H.form_q(V, tau)
    assert H.factor_backward_error(A, Q, R) < 10 * EPS * np.sqrt(m)
    assert H.orthogonality_error(Q) < 10 * EPS * np.sqrt(m) * np.sqrt(n)
    assert H.gram_error(A, R) < 10 * EPS * np.sqrt(m)
    z = np.random.default_rng(0).standard_normal(m)
    assert abs(np.linalg.norm(H.apply_qt(V, tau, z)) - np.linalg.norm(z)) < 50 * EPS * np.linalg.norm(z)


def _exact_ls(A, b):
    """Exact least-squares solution from the normal equations in rationals."""
    m, n = A.shape
    G = [[Fraction(int(sum(int(A[r, i]) * int(A[r, j]) for r in range(m)))) for j in range(n)] for i in range(n)]
    h = [Fraction(int(sum(int(A[r, i]) * int(b[r]) for r in range(m)))) for i in range(n)]
    for c in range(n):  # Gauss-Jordan, G is SPD so no pivoting is needed
        piv = G[c][c]
        for r in range(n):
            if r != c and G[r][c] != 0:
                f = G[r][c] / piv
                G[r] = [G[r][j] - f * G[c][j] for j in range(n)]
                h[r] -= f * h[c]
    return np.array([float(h[i] / G[i][i]) for i in range(n)])


@pytest.mark.parametrize("shape,seed", [((6, 3), 5), ((12, 4), 6), ((10, 10), 7)])
def test_lstsq_matches_exact_rational_solution(shape, seed):
    A = _int_matrix(*shape, seed)
    b = np.random.default_rng(seed).integers(-5, 6, size=shape[0]).astype(np.float64)
    x, R, qtb = H.lstsq(A, b)
    xe = _exact_ls(A, b)
    kappa = np.linalg.cond(A)
    assert np.abs(x - xe).max() <= 50 * kappa ** 2 * EPS * max(1.0, np.abs(xe).max())
    # residual norm equals the norm of the tail of Q^T b
    r = b - A @ x
    assert abs(np.linalg.norm(r) - np.linalg.norm(qtb[shape[1]:])) < 1e-12 * max(1, np.linalg.norm(b))


def test_backward_error_measures():
    A = synth.gaussian(300, 40, 1)
    b = synth.gaussian_rhs(300, 1, 1)[:, 0]
    x, _, _ = H.lstsq(A, b)
    assert H.ls_backward_error(A, b, x) < 50 * EPS
    x_bad = x + 1e-8
    assert H.ls_backward_error(A, b, x_bad) > 1e3 * EPS


def test_one_column_reflector_closed_form():
    """A single column x: R = -sign(x1) ||x||, and for x = e1 * a nothing changes."""
    x = np.array([3.0, 4.0])
    R, V, tau = H.qr(x[:, None])
    assert R[0, 0] == -5.0 and tau[0] == pytest.approx(1.6) and V[1, 0] == pytest.approx(0.5)
    R, V, tau = H.qr(np.array([[-2.0], [0.0], [0.0]]))
    assert R[0, 0] == -2.0 and tau[0] == 0.0
    R, V, tau = H.qr(np.array([[0.0], [2.0]]))
    assert R[0, 0] == -2.0  # sign(0) = +1


def test_planted_mistake_is_caught(monkeypatch):
    """Mutation check of the pins: a reflector with a dropped factor in tau
    (a plausible slip) must break the brute-force R pin."""
    good = H.reflector

    def bad(x):
        v, tau, beta = good(x)
        return v, tau * (1 + 1e-3), beta

    monkeypatch.setattr(H, "reflector", bad)
    A = _int_matrix(8, 3, 1)
    R, _, _ = H.qr(A)
    Rref = _chol_r_decimal(A)
    Ra, _ = H.row_sign_align(R, Rref)
    assert np.abs(Ra - Rref).max() / np.abs(Rref).max() > 1e-6
