"""Double-complex tiled QR on the GPU (the thesis's "z" workloads) against
the complex oracle: R (real diagonal, unique up to row signs for a
full-rank matrix), (Q^H b)(1:n), and the factorization's backward error
through the library's own Q^H, for every tree, both kernel families, nb 32
and 64, ragged shapes and one tile."""
import numpy as np
import pytest
import torch

import paper_1303_3182_amd as T
from oracle import zhouseholder as Z
from tests.gpu_util import EPS, case

pytestmark = pytest.mark.gpu


def _crandn(m, n, seed):
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n)))


def _check(A0, nb, tree, kernels, label):
    m, n = A0.shape
    o = T.default_opts(nb=nb, tree=tree, kernels=kernels)
    b0 = _crandn(m, 1, 99)
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    A, W = T.zfactor(T.zcolmajor(A0), o, info=info, nrhs=1)
    Bm = T.zcolmajor(b0)
    T.zapply_qh(A, W, Bm, o)
    torch.cuda.synchronize()
    assert int(info.item()) == 0, label
    R = np.triu(A.cpu().numpy()[:n, :n])
    Ro, Vo, tau = Z.zqr(A0)
    assert np.allclose(np.diag(R).imag, 0), label
    Ra, d = Z.row_sign_align(R, Ro)
    kap = np.linalg.cond(A0)
    tol = 2 * np.sqrt(2) * kap * 50 * EPS * np.linalg.norm(A0)
    assert np.linalg.norm(Ra - Ro) <= tol, (label, np.linalg.norm(Ra - Ro) / tol)
    c = Bm.cpu().numpy()[:n, 0] * d
    co = Z.zapply_qh(Vo, tau, b0[:, 0])[:n]
    assert np.linalg.norm(c - co) <= tol / np.linalg.norm(A0) * np.linalg.norm(b0), label
    # ||Q^H b|| = ||b|| (Q unitary)
    assert abs(np.linalg.norm(Bm.cpu().numpy()) - np.linalg.norm(b0)) <= 100 * EPS * np.linalg.norm(b0) * np.sqrt(m)


@pytest.mark.parametrize("nb", [32, 64])
def test_single_tile(nb):
    case("z single tile nb=%d" % nb)
    _check(_crandn(nb, nb, 1), nb, "greedy", "tt", "one tile")


@pytest.mark.parametrize("kernels", ["tt", "hybrid"])
@pytest.mark.parametrize("tree", ["flat", "binary", "fibonacci", "greedy", "grasap"])
def test_factor_matches_oracle(tree, kernels):
    for (m, n, nb) in [(256, 128, 64), (300, 170, 64), (200, 200, 32), (517, 77, 32)]:
        case("z factor %s %s m=%d n=%d nb=%d" % (tree, kernels, m, n, nb))
        _check(_crandn(m, n, m + n), nb, tree, kernels, (tree, kernels, m, n, nb))


def test_real_input_gives_the_real_factor():
    """A real matrix factored by the complex path gives the FP64 path's R
    (both follow the same reflector convention)."""
    case("z real input")
    rng = np.random.default_rng(5)
    A0 = np.asfortranarray(rng.standard_normal((320, 96)))
    o = T.default_opts(nb=64, tree="greedy")
    Az, _ = T.zfactor(T.zcolmajor(A0.astype(np.complex128)), o)
    Ar, _ = T.factor(T.colmajor(A0), T.default_opts(nb=64, ib=32, tree="greedy"))
    torch.cuda.synchronize()
    Rz = np.triu(Az.cpu().numpy()[:96, :96])
    Rr = np.triu(Ar.cpu().numpy()[:96, :96])
    assert np.abs(Rz.imag).max() <= 1e-12 * np.abs(Rz).max()
    assert np.linalg.norm(Rz.real - Rr) <= 1e-13 * np.linalg.norm(Rr)
