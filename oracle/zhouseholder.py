"""ORACLE -- test infrastructure only (see oracle/__init__).

Unblocked double-complex Householder QR, the factorization the thesis's
tiled algorithm computes on its double-complex ("z") workloads (chapter
"QR Factorization", section "Experimental results"): a sequence of unitary
reflections H_j = I - tau_j v_j v_j^H with H_n^H ... H_1^H A = R.

Reflector convention (the thesis fixes none; the GPU kernels use the same
one, so a one-tile factorization matches value for value): for
x = [alpha; x2], if x2 = 0 and alpha is real then tau = 0 (H = I);
otherwise beta = -sign(Re alpha) ||x|| (sign(0) = +1, beta real),
tau = (beta - alpha) / beta, v = [1; x2 / (alpha - beta)], and
H^H x = beta e1.  The diagonal of R is therefore real.
"""
import math

import numpy as np


def _norm2(x):
    """Euclidean norm of a complex vector, scaled against over/underflow."""
    x = np.asarray(x, dtype=np.complex128)
    if x.size == 0:
        return 0.0
    big = float(np.max(np.abs(x)))
    if big == 0.0 or not math.isfinite(big):
        return big
    y = x / big
    return big * math.sqrt(float(np.vdot(y, y).real))


def zreflector(x):
    """(v, tau, beta) of the reflector for the complex vector x."""
    x = np.asarray(x, dtype=np.complex128)
    alpha = complex(x[0])
    v = np.zeros_like(x)
    v[0] = 1.0
    if (x.size == 1 or float(np.max(np.abs(x[1:]))) == 0.0) and alpha.imag == 0.0:
        return v, 0j, alpha.real
    nrm = _norm2(x)
    beta = -nrm if alpha.real >= 0.0 else nrm
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def zqr(A):
    """Unblocked complex Householder QR of an m x n matrix (m >= n).

    Returns (R, V, tau): R n x n upper triangular with a real diagonal, V
    m x n unit lower trapezoidal, tau of length n.  Step j applies
    H_j^H = I - conj(tau_j) v_j v_j^H to the trailing columns."""
    A = np.array(A, dtype=np.complex128, order="F", copy=True)
    m, n = A.shape
    if m < n:
        raise ValueError("zqr needs m >= n")
    V = np.zeros((m, n), dtype=np.complex128)
    tau = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        v, t, beta = zreflector(A[j:, j])
        V[j:, j] = v
        tau[j] = t
        A[j, j] = beta
        A[j + 1:, j] = 0.0
        if t != 0 and j + 1 < n:
            w = v.conj() @ A[j:, j + 1:]
            A[j:, j + 1:] -= np.conj(t) * np.outer(v, w)
    return np.triu(A[:n, :]), V, tau


def zapply_qh(V, tau, B):
    """Q^H B = H_n^H ... H_1^H B."""
    B = np.array(B, dtype=np.complex128, copy=True)
    one = B.ndim == 1
    if one:
        B = B[:, None]
    for j in range(V.shape[1]):
        if tau[j] != 0:
            v = V[j:, j]
            B[j:] -= np.conj(tau[j]) * np.outer(v, v.conj() @ B[j:])
    return B[:, 0] if one else B


def zapply_q(V, tau, B):
    """Q B = H_1 ... H_n B."""
    B = np.array(B, dtype=np.complex128, copy=True)
    one = B.ndim == 1
    if one:
        B = B[:, None]
    for j in reversed(range(V.shape[1])):
        if tau[j] != 0:
            v = V[j:, j]
            B[j:] -= tau[j] * np.outer(v, v.conj() @ B[j:])
    return B[:, 0] if one else B


def row_sign_align(R_test, R_ref):
    """D R_test with D = diag(+-1) matching the (real) diagonals' signs."""
    d = np.sign(np.diag(R_test).real) * np.sign(np.diag(R_ref).real)
    d[d == 0] = 1.0
    return d[:, None] * R_test, d
