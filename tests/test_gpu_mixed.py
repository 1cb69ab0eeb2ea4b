"""Mixed precision: FP32 / BF16 MFMA trailing updates with FP64 panels, then
FP64 refinement, through the C ABI, against the FP64 oracle.

Bars:
- the low-precision factorization itself is backward stable to the update
  precision: ||Q^T A - [R; 0]||_F / ||A||_F <= c u_low (u = 2^-24 for FP32,
  2^-8 for BF16 with its 8-bit significand and FP32 accumulation), with
  c = 8 sqrt(n) (rounding of each of the O(q) block updates of every entry);
- after refinement the solution meets the FP64 bar: its normwise backward
  error, measured by the oracle in extended precision, is <= 50 eps
  (Stewart's bound for rectangular problems, Rigal-Gaches for square ones),
  and it agrees with the oracle's FP64 solution to the conditioning bound."""
import numpy as np
import pytest
import torch

import paper_1303_3182_amd as T
import synth
from oracle import householder as H
from tests.gpu_util import EPS, case

pytestmark = pytest.mark.gpu

U_LOW = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8}


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("kernels", ["tt", "hybrid"])
def test_low_precision_factor_backward_error(dtype, kernels):
    for (m, n, nb) in [(1024, 512, 128), (700, 300, 64), (512, 512, 256)]:
        case("mixed factor %s %s m=%d n=%d nb=%d" % (dtype, kernels, m, n, nb))
        A0 = synth.gaussian(m, n, 5 + m)
        o = T.default_opts(nb=nb, tree="greedy", kernels=kernels, update_dtype=dtype)
        A = T.colmajor(A0)
        A, W = T.factor(A, o, nrhs=n)
        Bm = T.colmajor(A0)
        T.apply_qt(A, W, Bm, o)   # FP64 replay of the stored reflectors
        torch.cuda.synchronize()
        R = np.triu(A.cpu().numpy()[:n])
        QtA = Bm.cpu().numpy()
        QtA[:n] -= R
        be = np.linalg.norm(QtA) / np.linalg.norm(A0)
        assert be <= 8 * np.sqrt(n) * U_LOW[dtype], (dtype, be)
        # and it is not the FP64 path in disguise: the error is well above FP64's
        assert be > 100 * EPS, (dtype, be)


def _lstsq(A0, B0, o):
    m, n = A0.shape
    nrhs = B0.shape[1]
    work = T.lstsq_workspace(m, n, nrhs, o)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    X = T.lstsq(T.colmajor(A0), T.colmajor(B0), o, work=work, info=info)
    torch.cuda.synchronize()
    return X.cpu().numpy(), int(info.item()), T.refine_report(work)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_refined_rectangular_least_squares(dtype):
    for (m, n, nb, nrhs) in [(1000, 300, 64, 1), (2048, 512, 128, 2), (3000, 257, 256, 1)]:
        case("mixed lstsq %s m=%d n=%d nb=%d nrhs=%d" % (dtype, m, n, nb, nrhs))
        A0 = synth.gaussian(m, n, 17 + m)
        B0 = synth.gaussian_rhs(m, nrhs, 17 + m)
        o = T.default_opts(nb=nb, tree="grasap", update_dtype=dtype, max_refine=20)
        X, info, rep = _lstsq(A0, B0, o)
        assert info == 0 and rep["done"] == 1, (info, rep)
        Ro, Vo, tau = H.qr(A0)
        QtB = H.apply_qt(Vo, tau, B0)
        kap = np.linalg.cond(A0)
        for c in range(nrhs):
            assert H.ls_backward_error(A0, B0[:, c], X[:, c]) <= 50 * EPS, rep
            xo = H.back_substitute(Ro, QtB[:n, c])
            assert np.linalg.norm(X[:, c] - xo) <= 100 * kap ** 2 * EPS * np.linalg.norm(xo)
        # refinement had work to do, and each step helped
        assert rep["iterations"] >= 1
        hist = rep["history"]
        assert hist[0] > 50 * EPS


@pytest.mark.parametrize("dtype,kappa", [("f32", 1e2), ("f32", 1e5), ("bf16", 1e2)])
def test_refined_square_conditioned(dtype, kappa):
    n, nb = 512, 128
    case("mixed square %s kappa=%g n=%d" % (dtype, kappa, n))
    A0, x0, b0 = synth.conditioned(n, kappa, 3)
    o = T.default_opts(nb=nb, tree="greedy", update_dtype=dtype, max_refine=20)
    X, info, rep = _lstsq(A0, b0[:, None], o)
    assert info == 0 and rep["done"] == 1, (info, rep)
    x = X[:, 0]
    assert H.ls_backward_error(A0, b0, x) <= 50 * EPS
    Ro, Vo, tau = H.qr(A0)
    xo = H.back_substitute(Ro, H.apply_qt(Vo, tau, b0)[:n])
    assert np.linalg.norm(x - xo) <= 100 * kappa * EPS * np.linalg.norm(xo)


@pytest.mark.parametrize("dtype,kappa", [("f32", 1e8)])
def test_gmres_refinement_where_classical_stalls(dtype, kappa):
    """kappa times the update precision's unit roundoff (2^-24 for FP32)
    above one: classical steps stall, and the AUTO method switches to GMRES
    preconditioned by the low-precision factors, which reaches the FP64
    bar."""
    n, nb = 1024, 128
    case("gmres refinement %s kappa=%g n=%d" % (dtype, kappa, n))
    A0, x0, b0 = synth.conditioned(n, kappa, 5)
    o = T.default_opts(nb=nb, tree="greedy", update_dtype=dtype, max_refine=20)
    X, info, rep = _lstsq(A0, b0[:, None], o)
    case("gmres refinement %s kappa=%g: report %s" % (dtype, kappa, rep))
    assert info == 0 and rep["done"] == 1, (info, rep)
    assert rep["gmres_steps"] >= 1 and rep["krylov_steps"] >= rep["gmres_steps"], rep
    x = X[:, 0]
    assert H.ls_backward_error(A0, b0, x) <= 50 * EPS
    Ro, Vo, tau = H.qr(A0)
    xo = H.back_substitute(Ro, H.apply_qt(Vo, tau, b0)[:n])
    assert np.linalg.norm(x - xo) <= 100 * kappa * EPS * np.linalg.norm(xo)
    # the classical method alone on the same system (reported, and never a
    # false pass: when it stops short, info says so)
    oc = T.default_opts(nb=nb, tree="greedy", update_dtype=dtype, max_refine=20, refine_method="classical")
    Xc, infoc, repc = _lstsq(A0, b0[:, None], oc)
    assert repc["gmres_steps"] == 0
    assert (infoc == 0) == (repc["done"] == 1) and (infoc in (0, -1001)), (infoc, repc)
    if infoc == 0:
        assert H.ls_backward_error(A0, b0, Xc[:, 0]) <= 50 * EPS


@pytest.mark.parametrize("kappa", [1e3, 1e4, 1e5])
def test_gmres_beyond_its_reach_is_reported(kappa):
    """BF16 updates (u_bf16 = 2^-8) at kappa 1e3..1e5: the factors may be
    too far from A for restarted GMRES(64) to converge.  Whatever happens,
    the outcome is reported truthfully: info 0 only with the FP64 bar met
    (checked by the oracle), else TQR_INFO_NOCONV with the measured error
    above the tolerance."""
    n, nb = 1024, 128
    case("gmres bf16 kappa=%g n=%d" % (kappa, n))
    A0, x0, b0 = synth.conditioned(n, kappa, 5)
    o = T.default_opts(nb=nb, tree="greedy", update_dtype="bf16", max_refine=6)
    X, info, rep = _lstsq(A0, b0[:, None], o)
    case("gmres bf16 kappa=%g: info %d report %s" % (kappa, info, rep))
    be = H.ls_backward_error(A0, b0, X[:, 0])
    if info == 0:
        assert rep["done"] == 1 and be <= 50 * EPS
    else:
        assert info == -1001 and rep["done"] == 0 and be > 16 * EPS and rep["backward_error"] > 16 * EPS


def test_gmres_method_from_the_first_step():
    n, nb = 700, 64
    case("gmres from the start n=%d" % n)
    A0, x0, b0 = synth.conditioned(n, 1e3, 6)
    o = T.default_opts(nb=nb, tree="fibonacci", update_dtype="f32", max_refine=10, refine_method="gmres")
    X, info, rep = _lstsq(A0, b0[:, None], o)
    assert info == 0 and rep["done"] == 1 and rep["gmres_steps"] == rep["iterations"] >= 1, rep
    assert H.ls_backward_error(A0, b0, X[:, 0]) <= 50 * EPS


def test_fp64_lstsq_report_untouched_by_refinement():
    A0 = synth.gaussian(300, 100, 1)
    B0 = synth.gaussian_rhs(300, 1, 1)
    X, info, rep = _lstsq(A0, B0, T.default_opts(nb=64))
    assert info == 0 and rep["done"] == 0 and rep["iterations"] == 0 and rep["history"] == []


def test_overflow_in_low_precision_updates_is_not_reported_as_success():
    """Entries near 2^126: the FP32 updates overflow and the factorization
    holds Inf / NaN.  The refinement must not call a NaN backward error a
    pass: the report stays not-done and info is TQR_INFO_NOCONV."""
    case("f32 overflow")
    A0 = synth.gaussian(600, 200, 8) * 2.0 ** 126
    B0 = synth.gaussian_rhs(600, 1, 8) * 2.0 ** 126
    o = T.default_opts(nb=64, tree="greedy", update_dtype="f32", max_refine=3)
    X, info, rep = _lstsq(A0, B0, o)
    assert rep["done"] == 0, rep
    assert info == -1001, info  # TQR_INFO_NOCONV
    assert not (rep["backward_error"] <= 16 * EPS), rep
