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


# ------------------------------------------------ exact pins of the measures

def _dec_sqrt(fr, digits=50):
    getcontext().prec = digits
    return (Decimal(fr.numerator) / Decimal(fr.denominator)).sqrt()


def _exact_stewart(A, b, x):
    """||A^T r|| / (||A||_F ||r||), r = b - A x, from the exact rational
    values of the float64 inputs (Fraction) with 50-digit square roots."""
    m, n = A.shape
    Af = [[Fraction(float(A[i, j])) for j in range(n)] for i in range(m)]
    xf = [Fraction(float(v)) for v in x]
    r = [Fraction(float(b[i])) - sum(Af[i][j] * xf[j] for j in range(n)) for i in range(m)]
    atr = [sum(Af[i][j] * r[i] for i in range(m)) for j in range(n)]
    num = _dec_sqrt(sum(v * v for v in atr))
    den = _dec_sqrt(sum(v * v for row in Af for v in row)) * _dec_sqrt(sum(v * v for v in r))
    return float(num / den)


def _exact_rigal_gaches(A, b, x):
    """||b - A x|| / (||A||_F ||x|| + ||b||), exactly (square branch)."""
    n = A.shape[0]
    Af = [[Fraction(float(A[i, j])) for j in range(n)] for i in range(n)]
    xf = [Fraction(float(v)) for v in x]
    bf = [Fraction(float(v)) for v in b]
    r = [bf[i] - sum(Af[i][j] * xf[j] for j in range(n)) for i in range(n)]
    num = _dec_sqrt(sum(v * v for v in r))
    den = (_dec_sqrt(sum(v * v for row in Af for v in row)) * _dec_sqrt(sum(v * v for v in xf))
           + _dec_sqrt(sum(v * v for v in bf)))
    return float(num / den)


def test_stewart_bound_matches_exact_value():
    """Rectangular branch of ls_backward_error against its definition in
    exact arithmetic, for an x far from the solution and for the float64
    rounding of the exact solution (there A^T r is of order eps: a float64
    evaluation of the measure would be wrong in its leading digit, the
    extended-precision one keeps several)."""
    A = _int_matrix(7, 3, 21)
    b = np.random.default_rng(21).integers(-6, 7, size=7).astype(np.float64)
    xe = _exact_ls(A, b)
    for x, rtol in [(xe + np.array([0.25, -0.375, 0.125]), 1e-12), (xe * (1 + 3e-9), 1e-9), (xe, 1e-3)]:
        got = H.ls_backward_error(A, b, x)
        want = _exact_stewart(A, b, x)
        assert want > 0
        assert abs(got - want) <= rtol * want, (got, want)
    assert _exact_stewart(A, b, xe) < 10 * EPS


def test_rigal_gaches_matches_exact_value():
    A = _int_matrix(5, 5, 22)
    b = np.random.default_rng(22).integers(-6, 7, size=5).astype(np.float64)
    xe = _exact_ls(A, b)
    for x, rtol in [(xe + 0.0625, 1e-12), (xe, 1e-3)]:
        got = H.ls_backward_error(A, b, x)
        want = _exact_rigal_gaches(A, b, x)
        assert abs(got - want) <= rtol * want, (got, want)


def test_gram_error_matches_exact_value():
    """gram_error against its definition evaluated exactly (same probes),
    for a correct R and for R with one planted error."""
    A = _int_matrix(6, 3, 23)
    Rok = _chol_r_decimal(A)
    Rbad = Rok.copy()
    Rbad[0, 2] += 1e-6
    Z = H.gram_probes(3, 8, 0)
    # (near eps the measure is a cancellation: long double keeps ~3 digits)
    for R, rtol in ((Rok, 1e-3), (Rbad, 1e-9)):
        worst = Decimal(0)
        Af = [[Fraction(float(A[i, j])) for j in range(3)] for i in range(6)]
        Rf = [[Fraction(float(R[i, j])) for j in range(3)] for i in range(3)]
        for c in range(Z.shape[1]):
            z = [Fraction(float(v)) for v in Z[:, c]]
            az = [sum(Af[i][j] * z[j] for j in range(3)) for i in range(6)]
            g = [sum(Af[i][j] * az[i] for i in range(6)) for j in range(3)]
            rz = [sum(Rf[i][j] * z[j] for j in range(3)) for i in range(3)]
            h = [sum(Rf[i][j] * rz[i] for i in range(3)) for j in range(3)]
            e = _dec_sqrt(sum((h[j] - g[j]) ** 2 for j in range(3))) / _dec_sqrt(sum(v * v for v in g))
            worst = max(worst, e)
        got = H.gram_error(A, R)
        assert abs(got - float(worst)) <= rtol * float(worst), (got, worst)
    assert H.gram_error(A, Rok) < 20 * EPS
    assert H.gram_error(A, Rbad) > 1e-8


def test_gram_error_catches_one_wrong_entry_at_scale():
    """A backward-stable R of a tall Gaussian matrix sits near eps; one entry
    off by 1e-8 ||A||_F is caught by many orders of magnitude."""
    A = synth.gaussian(2000, 300, 24)
    R, _, _ = H.qr(A)
    assert H.gram_error(A, R) < 50 * EPS
    Rb = R.copy()
    Rb[150, 280] += 1e-8 * np.linalg.norm(A)
    assert H.gram_error(A, Rb) > 1e4 * 50 * EPS


def test_factor_and_orthogonality_measures_exact():
    """||A - QR||_F / ||A||_F and ||Q^T Q - I||_F on hand-computable inputs."""
    A = np.array([[3.0, 0.0], [4.0, 0.0], [0.0, 2.0]])
    Q = np.array([[0.6, 0.0], [0.8, 0.0], [0.0, 1.0]])
    R = np.array([[5.0, 0.0], [0.0, 2.0]])
    assert H.factor_backward_error(A, Q, R) == pytest.approx(0.0, abs=1e-16)
    R2 = np.array([[5.0, 0.0], [0.0, 4.0]])  # error 2 in the last column: ||[0,0,-2]|| / sqrt(29)
    assert H.factor_backward_error(A, Q, R2) == pytest.approx(2.0 / np.sqrt(29.0), rel=1e-15)
    assert H.orthogonality_error(2.0 * np.eye(3)) == pytest.approx(np.sqrt(27.0), rel=1e-15)


@pytest.mark.parametrize("s", [530, -530])
def test_extreme_scaling_is_exact(s):
    """Entries near the overflow (2^530 ~ 1e160) or underflow (2^-530 ~
    1e-160) threshold: the squares in ||x|| would overflow / underflow, the
    scaled norm does not, and scaling A by a power of two scales R exactly.
    The least-squares measure stays finite and scale invariant."""
    A = synth.gaussian(40, 17, 31)
    b = synth.gaussian_rhs(40, 1, 31)[:, 0]
    R1, V1, t1 = H.qr(A)
    R2, V2, t2 = H.qr(A * 2.0 ** s)
    assert np.array_equal(R2, R1 * 2.0 ** s)
    assert np.array_equal(V2, V1) and np.array_equal(t2, t1)
    x1, _, _ = H.lstsq(A, b)
    x2, _, _ = H.lstsq(A * 2.0 ** s, b * 2.0 ** s)
    assert np.array_equal(x1, x2)
    e1, e2 = H.ls_backward_error(A, b, x1), H.ls_backward_error(A * 2.0 ** s, b * 2.0 ** s, x2)
    assert np.isfinite(e2) and abs(e1 - e2) <= 1e-6 * e1


def test_unscaled_norm_is_a_caught_mistake(monkeypatch):
    """Planted mistake: the reflector's norm formed from unscaled squares.
    At 2^530 it overflows; the exact-scaling pin must catch it."""
    def unscaled(x):
        x = np.asarray(x, dtype=np.float64)
        with np.errstate(over="ignore", under="ignore"):
            return float(np.sqrt(np.dot(x, x)))
    monkeypatch.setattr(H, "_norm2", unscaled)
    A = synth.gaussian(40, 17, 31)
    with np.errstate(all="ignore"):
        R2, _, _ = H.qr(A * 2.0 ** 530)
    R1, _, _ = H.qr(A)
    assert not np.array_equal(R2, R1 * 2.0 ** 530)


def test_planted_measure_mistakes_are_caught(monkeypatch):
    """Mutations of the two measures (scaled by 0.01, or a constant 0) must
    fail the exact pins above."""
    A = _int_matrix(7, 3, 21)
    b = np.random.default_rng(21).integers(-6, 7, size=7).astype(np.float64)
    x = _exact_ls(A, b) + np.array([0.25, -0.375, 0.125])
    want = _exact_stewart(A, b, x)
    good_be, good_ge = H.ls_backward_error, H.gram_error
    monkeypatch.setattr(H, "ls_backward_error", lambda *a: 0.01 * good_be(*a))
    assert abs(H.ls_backward_error(A, b, x) - want) > 1e-12 * want
    Rbad = _chol_r_decimal(A)
    Rbad[0, 2] += 1e-6
    monkeypatch.setattr(H, "gram_error", lambda *a, **k: 0.0)
    assert not H.gram_error(A, Rbad) > 1e-8
    monkeypatch.setattr(H, "gram_error", good_ge)
    assert H.gram_error(A, Rbad) > 1e-8
