"""Tile Cholesky inversion on the GPU (chapter "Cholesky Inversion",
algorithm alg:InPlace) against the oracle's unblocked inverse, element by
element: both are backward stable, so they agree to a few kappa(A) eps
||A^{-1}||.  Covers both variants (in place, array renaming), both loop
orders, nb 32 and 64, ragged sizes, one tile, and a matrix that is not
positive definite (info reports the leading minor)."""
import numpy as np
import pytest
import torch

import paper_1303_3182_amd as T
from oracle import cholinv as C
from tests.gpu_util import EPS, case

pytestmark = pytest.mark.gpu


def _spd(n, seed, kappa=None):
    rng = np.random.default_rng(seed)
    if kappa is None:
        G = rng.standard_normal((n, n))
        return G @ G.T / n + np.eye(n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = kappa ** (-np.arange(n) / max(n - 1, 1))
    return (Q * s) @ Q.T


def _run(A0, nb, variant):
    n = A0.shape[0]
    A = T.colmajor(A0)
    upper = torch.triu(A, 1).clone()
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    T.cholinv(A, nb=nb, variant=variant, info=info)
    torch.cuda.synchronize()
    assert torch.equal(torch.triu(A, 1), upper)  # the strict upper triangle is not touched
    return np.tril(A.cpu().numpy()), int(info.item())


@pytest.mark.parametrize("variant", [T.CHOLINV_INPLACE, T.CHOLINV_RENAMED, T.CHOLINV_UUU,
                                     T.CHOLINV_RENAMED | T.CHOLINV_UUU])
@pytest.mark.parametrize("nb", [32, 64])
def test_cholinv_matches_oracle(nb, variant):
    for (n, seed, kappa) in [(1, 1, None), (nb, 2, None), (3 * nb + 7, 3, None), (300, 4, 1e4), (517, 5, None)]:
        case("cholinv nb=%d variant=%d n=%d" % (nb, variant, n))
        A0 = _spd(n, seed, kappa)
        X, info = _run(A0, nb, variant)
        assert info == 0
        Xo = np.tril(C.spd_inverse(A0))
        kap = np.linalg.cond(A0)
        assert np.linalg.norm(X - Xo) <= 8 * n * kap * EPS * np.linalg.norm(Xo), (n, np.linalg.norm(X - Xo))


def test_cholinv_not_positive_definite():
    n, nb = 200, 64
    A0 = _spd(n, 7)
    A0[150, 150] = -5.0  # the leading minor of order 151 is not positive definite
    case("cholinv not positive definite")
    _, info = _run(A0, nb, T.CHOLINV_INPLACE)
    assert info == 151
