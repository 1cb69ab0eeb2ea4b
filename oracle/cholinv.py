"""ORACLE -- test infrastructure only (see oracle/__init__).

Inverse of a symmetric positive definite matrix through its Cholesky
factor, as the thesis's chapter "Cholesky Inversion" defines it (algorithm
alg:InPlace, its three steps): A = L L^T (step 1), W = L^{-1} (step 2),
A^{-1} = W^T W (step 3).  Written from those definitions, unblocked and in
FP64, with no tiling, blocking or reordering; the tiled algorithm reaches
the same result up to rounding order.
"""
import numpy as np


def cholesky(A):
    """Lower-triangular L with L L^T = A, column by column:
    L[j,j] = sqrt(A[j,j] - sum_{k<j} L[j,k]^2),
    L[i,j] = (A[i,j] - sum_{k<j} L[i,k] L[j,k]) / L[j,j] for i > j."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.zeros((n, n))
    for j in range(n):
        d = A[j, j] - L[j, :j] @ L[j, :j]
        if not d > 0.0:
            raise np.linalg.LinAlgError("matrix is not positive definite (column %d)" % j)
        L[j, j] = np.sqrt(d)
        L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L


def lower_inverse(L):
    """W = L^{-1} for lower-triangular L: column c of W solves L w = e_c by
    forward substitution (w is zero above row c)."""
    L = np.asarray(L, dtype=np.float64)
    n = L.shape[0]
    W = np.zeros((n, n))
    for c in range(n):
        w = np.zeros(n)
        w[c] = 1.0 / L[c, c]
        for i in range(c + 1, n):
            w[i] = -(L[i, c:i] @ w[c:i]) / L[i, i]
        W[:, c] = w
    return W


def spd_inverse(A):
    """A^{-1} = W^T W with W = L^{-1}, L the Cholesky factor of A
    (returned full and symmetric)."""
    W = lower_inverse(cholesky(A))
    X = W.T @ W
    return np.tril(X) + np.tril(X, -1).T
