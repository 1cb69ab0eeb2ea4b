"""Pins of the double-complex Householder oracle (oracle/zhouseholder.py):

* the reflector's defining property H^H x = beta e1 with H unitary;
* real input reduces to the real oracle (oracle/householder.py);
* R^H R = A^H A against the Cholesky factor of A^H A computed in 50-digit
  arithmetic (mpmath), the unique R with a positive diagonal;
* A = Q R with Q^H Q = I (Q formed from the reflectors);
* special cases: an upper-triangular input with a real diagonal is its own
  R (every tau is 0), a complex diagonal input gives R = diag(-sign(Re d)|d|);
* a planted mistake (tau instead of conj(tau) when applying H^H) fails."""
import mpmath
import numpy as np

from oracle import householder as H
from oracle import zhouseholder as Z

EPS = np.finfo(np.float64).eps


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_reflector_definition():
    rng = np.random.default_rng(1)
    for n in (1, 2, 5, 40):
        x = _crandn(rng, n)
        v, tau, beta = Z.zreflector(x)
        Hm = np.eye(n) - tau * np.outer(v, v.conj())
        assert np.allclose(Hm.conj().T @ Hm, np.eye(n), atol=20 * EPS)
        y = Hm.conj().T @ x
        assert abs(y[0] - beta) <= 20 * EPS * np.linalg.norm(x)
        assert np.linalg.norm(y[1:]) <= 20 * EPS * np.linalg.norm(x)
        assert abs(beta) == np.float64(abs(beta)) and isinstance(beta, float)


def test_real_input_matches_real_oracle():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((30, 12))
    Rz, _, tz = Z.zqr(A)
    Rr, _, tr = H.qr(A)
    assert np.allclose(Rz.imag, 0)
    assert np.allclose(Rz.real, Rr, atol=10 * EPS * np.linalg.norm(A))
    assert np.allclose(tz, tr, atol=10 * EPS)


def test_gram_against_50_digit_cholesky():
    rng = np.random.default_rng(3)
    mpmath.mp.dps = 50
    for (m, n) in [(6, 3), (9, 5), (12, 8)]:
        A = _crandn(rng, m, n)
        Am = mpmath.matrix([[mpmath.mpc(A[i, j].real, A[i, j].imag) for j in range(n)] for i in range(m)])
        G = Am.H * Am
        L = mpmath.zeros(n, n)
        for j in range(n):
            s = G[j, j] - sum(abs(L[j, k]) ** 2 for k in range(j))
            L[j, j] = mpmath.sqrt(mpmath.re(s))
            for i in range(j + 1, n):
                L[i, j] = (G[i, j] - sum(L[i, k] * mpmath.conj(L[j, k]) for k in range(j))) / L[j, j]
        Rref = np.array([[complex(mpmath.conj(L[j, i])) for j in range(n)] for i in range(n)])  # L^H
        R, _, _ = Z.zqr(A)
        Ra, _ = Z.row_sign_align(R, Rref)
        kap = np.linalg.cond(A)
        assert np.linalg.norm(Ra - Rref) <= 10 * kap * EPS * np.linalg.norm(A), (m, n)


def test_factorization_and_unitarity():
    rng = np.random.default_rng(4)
    A = _crandn(rng, 50, 20)
    R, V, tau = Z.zqr(A)
    Q = Z.zapply_q(V, tau, np.eye(50, 20))
    assert np.linalg.norm(Q.conj().T @ Q - np.eye(20)) <= 50 * EPS
    assert np.linalg.norm(A - Q @ R) <= 50 * EPS * np.linalg.norm(A)
    QhA = Z.zapply_qh(V, tau, A)
    assert np.linalg.norm(QhA[:20] - R) <= 50 * EPS * np.linalg.norm(A)
    assert np.linalg.norm(QhA[20:]) <= 50 * EPS * np.linalg.norm(A)
    assert np.allclose(np.diag(R).imag, 0)


def test_special_cases():
    rng = np.random.default_rng(5)
    T = np.triu(_crandn(rng, 7, 7))
    T[np.diag_indices(7)] = rng.standard_normal(7)
    R, V, tau = Z.zqr(T)
    assert np.all(tau == 0) and np.array_equal(R, T)
    d = _crandn(rng, 6)
    R, _, _ = Z.zqr(np.diag(d))
    expect = np.diag(np.where(d.real >= 0, -1.0, 1.0) * np.abs(d))
    assert np.allclose(R, expect, atol=4 * EPS * np.abs(d).max())


def test_planted_mistake_is_caught():
    """Applying I - tau v v^H instead of H^H = I - conj(tau) v v^H."""
    rng = np.random.default_rng(6)
    A = _crandn(rng, 10, 6)
    R, _, _ = Z.zqr(A)
    B = np.array(A, copy=True)
    for j in range(6):
        v, t, beta = Z.zreflector(B[j:, j])
        B[j, j] = beta
        B[j + 1:, j] = 0
        B[j:, j + 1:] -= t * np.outer(v, v.conj() @ B[j:, j + 1:])
    Rw = np.triu(B[:6])
    G = A.conj().T @ A
    assert np.linalg.norm(R.conj().T @ R - G) <= 100 * EPS * np.linalg.norm(G)
    assert np.linalg.norm(Rw.conj().T @ Rw - G) > 1e-6 * np.linalg.norm(G)
