"""ORACLE -- test infrastructure only (see oracle/__init__).

Unblocked FP64 Householder QR, written from the textbook definition the
thesis builds on (chapter "QR Factorization", introduction: a sequence of
orthogonal transformations U_l ... U_1 A = R, each Householder reflection
zeroing the entries below the diagonal of one column; the tiled algorithm
reaches exactly this R factor with the same flop count 2mn^2 - 2n^3/3,
theorem thm.flops).

Reflector convention (the thesis fixes none; the same convention is used
by the GPU kernels so that a one-tile factorization matches sign for sign):
for x = [alpha; x2], if ||x2|| = 0 then tau = 0 and H = I; otherwise
beta = -sign(alpha) ||x|| with sign(0) = +1, tau = (beta - alpha) / beta and
v = [1; x2 / (alpha - beta)], H = I - tau v v^T, H x = beta e1.
"""
import math

import numpy as np


def _norm2(x):
    """Euclidean norm without overflow or underflow in the squares: the
    entries are divided by the largest magnitude first (so every square is
    at most 1) and the result is scaled back."""
    x = np.asarray(x, dtype=np.float64)
    if x.size == 0:
        return 0.0
    big = float(np.max(np.abs(x)))
    if big == 0.0 or not math.isfinite(big):
        return big
    y = x / big
    return big * math.sqrt(float(np.dot(y, y)))


def reflector(x):
    """(v, tau, beta) of the Householder reflector for the vector x.

    ||x|| is formed with scaling (_norm2), so entries near the overflow or
    underflow threshold give the same reflector as the scaled vector."""
    x = np.asarray(x, dtype=np.float64)
    alpha = float(x[0])
    v = np.zeros_like(x)
    v[0] = 1.0
    if x.size == 1 or float(np.max(np.abs(x[1:]))) == 0.0:
        return v, 0.0, alpha
    norm = _norm2(x)
    beta = -norm if alpha >= 0.0 else norm
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def qr(A):
    """Unblocked Householder QR of an m x n matrix (m >= n).

    Returns (R, V, tau): R is n x n upper triangular, V is m x n unit lower
    trapezoidal (column j holds the reflector of step j), tau has n entries.
    Each step applies its reflector to the trailing columns only."""
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    m, n = A.shape
    if m < n:
        raise ValueError("qr needs m >= n")
    V = np.zeros((m, n))
    tau = np.zeros(n)
    for j in range(n):
        v, t, beta = reflector(A[j:, j])
        V[j:, j] = v
        tau[j] = t
        A[j, j] = beta
        A[j + 1:, j] = 0.0
        if t != 0.0 and j + 1 < n:
            w = v @ A[j:, j + 1:]
            A[j:, j + 1:] -= t * np.outer(v, w)
    return np.triu(A[:n, :]), V, tau


def apply_qt(V, tau, B):
    """Q^T B with Q = H_1 H_2 ... H_n, i.e. H_n ... H_1 B."""
    B = np.array(B, dtype=np.float64, copy=True)
    one = B.ndim == 1
    if one:
        B = B[:, None]
    for j in range(V.shape[1]):
        if tau[j] != 0.0:
            v = V[j:, j]
            B[j:] -= tau[j] * np.outer(v, v @ B[j:])
    return B[:, 0] if one else B


def apply_q(V, tau, B):
    """Q B = H_1 ... H_n B."""
    B = np.array(B, dtype=np.float64, copy=True)
    one = B.ndim == 1
    if one:
        B = B[:, None]
    for j in reversed(range(V.shape[1])):
        if tau[j] != 0.0:
            v = V[j:, j]
            B[j:] -= tau[j] * np.outer(v, v @ B[j:])
    return B[:, 0] if one else B


def form_q(V, tau):
    """The m x n matrix Q with orthonormal columns (A = Q R)."""
    m, n = V.shape
    return apply_q(V, tau, np.eye(m, n))


def back_substitute(R, c):
    """Solve R x = c for upper-triangular R, one row at a time from the bottom."""
    R = np.asarray(R, dtype=np.float64)
    c = np.array(c, dtype=np.float64, copy=True)
    one = c.ndim == 1
    if one:
        c = c[:, None]
    n = R.shape[0]
    x = np.zeros((n, c.shape[1]))
    for i in range(n - 1, -1, -1):
        x[i] = (c[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    return x[:, 0] if one else x


def lstsq(A, B):
    """Least squares min ||A x - b|| via R x = (Q^T b)_{1:n}.

    Returns (x, R, qtb) where qtb is the full Q^T b (its tail norm is the
    residual norm)."""
    A = np.asarray(A, dtype=np.float64)
    R, V, tau = qr(A)
    qtb = apply_qt(V, tau, B)
    n = A.shape[1]
    x = back_substitute(R, qtb[:n])
    return x, R, qtb


# --------------------------------------------------------------- measures

def row_sign_align(R_test, R_ref):
    """D = sign(diag R_test) * sign(diag R_ref); returns D R_test (R is unique
    up to D = diag(+-1) for a full-rank A)."""
    d = np.sign(np.diag(R_test)) * np.sign(np.diag(R_ref))
    d[d == 0] = 1.0
    return d[:, None] * R_test, d


def factor_backward_error(A, Q, R):
    """||A - Q R||_F / ||A||_F."""
    return np.linalg.norm(A - Q @ R) / np.linalg.norm(A)


def orthogonality_error(Q):
    """||Q^T Q - I||_F."""
    return np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1]))


def gram_probes(n, probes=8, seed=0):
    """The Gaussian probe vectors gram_error uses (n x probes)."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.standard_normal(n) for _ in range(probes)], axis=1)


def gram_error(A, R, probes=8, seed=0):
    """Randomised check of R^T R = A^T A: the largest relative error
    ||R^T (R z) - A^T (A z)|| / ||A^T (A z)|| over Gaussian probes z.

    The normalisation is the natural scale of the Gram action (about
    ||A||_2^2 ||z||), so a backward-stable R gives a value of a few eps.
    Both products are formed in extended precision (long double) so that
    their own rounding does not mask an error of that size."""
    Al = np.asarray(A, dtype=np.float64).astype(np.longdouble)
    Rl = np.asarray(R, dtype=np.float64).astype(np.longdouble)
    Z = gram_probes(Al.shape[1], probes, seed).astype(np.longdouble)
    worst = 0.0
    for c in range(Z.shape[1]):
        z = Z[:, c]
        g = Al.T @ (Al @ z)
        d = Rl.T @ (Rl @ z) - g
        e = float(np.sqrt(np.dot(d, d)) / np.sqrt(np.dot(g, g)))
        worst = max(worst, e)
    return worst


def ls_backward_error(A, b, x):
    """Normwise backward-error bound for a least-squares solution.

    Square systems: Rigal-Gaches ||b - A x|| / (||A||_F ||x|| + ||b||).
    Rectangular: Stewart's one-sided bound ||A^T r|| / (||A||_F ||r||) with
    r = b - A x (x is the exact LS solution of a problem perturbed by
    E = -r r^T A / ||r||^2, ||E||_2 = ||A^T r|| / ||r||).  Every product
    and norm is formed in extended precision (long double, also wide enough
    in exponent for entries near the FP64 overflow threshold) so that the
    measure's own rounding does not mask errors of order 50 eps."""
    Al = np.asarray(A, dtype=np.float64).astype(np.longdouble)
    bl = np.asarray(b, dtype=np.float64).astype(np.longdouble)
    xl = np.asarray(x, dtype=np.float64).astype(np.longdouble)
    r = bl - Al @ xl
    nA = np.sqrt(np.sum(Al * Al))
    nr = np.sqrt(np.dot(r, r))
    if Al.shape[0] == Al.shape[1]:
        return float(nr / (nA * np.sqrt(np.dot(xl, xl)) + np.sqrt(np.dot(bl, bl))))
    if nr == 0:
        return 0.0
    atr = Al.T @ r
    return float(np.sqrt(np.dot(atr, atr)) / (nA * nr))
