"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module only draws random numbers and shapes; it holds none of the QR
method's arithmetic.  Matrices are float64 in column-major (Fortran) order,
generated on the CPU with numpy's PCG64 so that the oracle and the GPU path
see identical bits.

The thesis's experiments do not state their matrix entry distribution; the
workloads below follow the sizes it and the project name (i.i.d. N(0,1)
entries, prescribed-condition square systems, ragged batches).
"""
import functools
import math

import numpy as np


def gaussian(m, n, seed):
    """m x n matrix of i.i.d. N(0,1) entries, column-major float64."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((m, n)))


def gaussian_rhs(m, nrhs, seed):
    rng = np.random.default_rng(seed + 0x5EED)
    return np.asfortranarray(rng.standard_normal((m, nrhs)))


@functools.lru_cache(maxsize=4)
def _haar_cached(n, seed):
    return haar_orthogonal(n, seed)


def haar_orthogonal(n, seed):
    """Haar-distributed orthogonal matrix: the Q of a Gaussian matrix's QR
    with its columns multiplied by sign(diag R) (input synthesis only)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def conditioned(n, kappa, seed):
    """A = U diag(sigma) V^T with Haar U, V and sigma_i = kappa^(-(i-1)/(n-1)).

    Returns (A, x, b) with x ~ N(0,1) and b = A x + 1e-6 N(0,1)."""
    U = _haar_cached(n, seed)
    Vt = _haar_cached(n, seed + 1).T
    i = np.arange(n, dtype=np.float64)
    sigma = kappa ** (-i / max(n - 1, 1))
    A = np.asfortranarray((U * sigma[None, :]) @ Vt)
    rng = np.random.default_rng(seed + 2)
    x = rng.standard_normal(n)
    b = A @ x + 1e-6 * rng.standard_normal(n)
    return A, x, b


def ragged_batch_shapes(count, seed, m_range=(256, 8192), n_range=(32, 512)):
    """Shapes of a ragged least-squares batch: m and n log-uniform in their
    ranges, rejecting n > m/2."""
    rng = np.random.default_rng(seed)
    shapes = []
    while len(shapes) < count:
        m = int(round(math.exp(rng.uniform(math.log(m_range[0]), math.log(m_range[1])))))
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        if n <= m // 2:
            shapes.append((m, n))
    return shapes


def ragged_batch(shapes, seed, nrhs=1):
    """Matrices and right-hand sides of a ragged batch, i.i.d. N(0,1):
    lists As (m x n) and Bs (m x nrhs), column-major, one generator stream
    per problem."""
    As, Bs = [], []
    for idx, (m, n) in enumerate(shapes):
        rng = np.random.default_rng([seed, idx])
        As.append(np.asfortranarray(rng.standard_normal((m, n))))
        Bs.append(np.asfortranarray(rng.standard_normal((m, nrhs))))
    return As, Bs
