"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (square systems: nb 128, ib 32, PlasmaTree with TS
domains of 48 tile rows merged by TT kernels; persistent executor in the
static list order).

Square 8192 x 8192 systems with prescribed condition number (A = U diag(s)
V^T, Haar U and V, log-spaced s; b = A x + 1e-6 N(0,1)):
- R(:, 1:nb) and (Q^T b)(1:nb) depend only on the first tile column and
  its FP64 panel kernels, so they are compared elementwise with the oracle's
  factorization of A(:, 1:256), for every update precision (the
  low-precision updates touch later tile columns only);
- the solution (FP64, or refined after FP32 / BF16 updates) must meet the
  FP64 bar: normwise backward error (Rigal-Gaches, by the oracle in
  extended precision) <= 50 eps.
FP32 at kappa 1e8 (kappa u_fp32 ~ 6 before the growth of the factorization
error with n): classical steps stall and the GMRES-based steps do not
reach the bar at this size; the outcome must be reported truthfully.
Ragged least-squares batch at the ranges of the batched workload (m up to
8192, n up to 512): every member's backward error (Stewart's bound) <= 50 eps
and, for a sample of members, x against the oracle's x."""
import numpy as np
import pytest
import torch

import paper_1303_3182_amd as T
import synth
from oracle import householder as H
from tests.gpu_util import EPS, case, r_tol

pytestmark = pytest.mark.gpu

N, NB = 8192, 128
SQ = dict(nb=NB, ib=32, tree="plasma", param=48, kernels="hybrid")


def _first_column_oracle(A0, b0):
    Ro, Vo, tau = H.qr(A0[:, :NB])
    return Ro, H.apply_qt(Vo, tau, b0)[:NB]


@pytest.mark.parametrize("dtype,kappa", [("f64", 1e5), ("f32", 1e5), ("bf16", 1e2)])
def test_square_8192(dtype, kappa):
    case("square 8192 %s kappa=%g: inputs" % (dtype, kappa))
    A0, x0, b0 = synth.conditioned(N, kappa, 7)
    o = T.default_opts(update_dtype=dtype, max_refine=20, **SQ)
    case("square 8192 %s kappa=%g: factor + Q^T b" % (dtype, kappa))
    A, W = T.factor(T.colmajor(A0), o, nrhs=1)
    Bm = T.colmajor(b0[:, None])
    T.apply_qt(A, W, Bm, o)
    torch.cuda.synchronize()
    R1 = np.triu(A[:NB, :NB].cpu().numpy())
    c1 = Bm[:NB, 0].cpu().numpy()
    del A, W
    Ro, co = _first_column_oracle(A0, b0)
    Ra, d = H.row_sign_align(R1, Ro)
    tol = r_tol(A0[:, :NB])
    assert np.linalg.norm(Ra - Ro) <= tol
    assert np.linalg.norm(c1 * d - co) <= tol / np.linalg.norm(A0[:, :NB]) * np.linalg.norm(b0)
    case("square 8192 %s kappa=%g: lstsq" % (dtype, kappa))
    work = T.lstsq_workspace(N, N, 1, o)
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    X = T.lstsq(T.colmajor(A0), T.colmajor(b0[:, None]), o, work=work, info=info)
    torch.cuda.synchronize()
    rep = T.refine_report(work)
    assert int(info.item()) == 0, (int(info.item()), rep)
    be = H.ls_backward_error(A0, b0, X[:, 0].cpu().numpy())
    assert be <= 50 * EPS, (be / EPS, rep)
    if dtype != "f64":
        assert rep["done"] == 1 and rep["iterations"] >= 1, rep


def test_square_8192_fp32_kappa_1e8_is_reported():
    A0, x0, b0 = synth.conditioned(N, 1e8, 7)
    o = T.default_opts(update_dtype="f32", max_refine=20, **SQ)
    case("square 8192 f32 kappa=1e8: lstsq")
    work = T.lstsq_workspace(N, N, 1, o)
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    X = T.lstsq(T.colmajor(A0), T.colmajor(b0[:, None]), o, work=work, info=info)
    torch.cuda.synchronize()
    rep = T.refine_report(work)
    case("square 8192 f32 kappa=1e8: report %s" % rep)
    be = H.ls_backward_error(A0, b0, X[:, 0].cpu().numpy())
    assert rep["gmres_steps"] >= 1  # classical steps stalled and GMRES was tried
    if int(info.item()) == 0:
        assert rep["done"] == 1 and be <= 50 * EPS
    else:
        assert int(info.item()) == -1001 and rep["done"] == 0 and be > 16 * EPS


def _batch_c4(count, seed):
    shapes = synth.ragged_batch_shapes(count, seed)
    As, Bs = synth.ragged_batch(shapes, seed, 1)
    return shapes, As, Bs


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batched_full_ranges(dtype):
    shapes, As, Bs = _batch_c4(64, 1)
    case("batched 64 %s, m<=%d n<=%d" % (dtype, max(m for m, _ in shapes), max(n for _, n in shapes)))
    o = T.default_opts(nb=128, ib=32, tree="auto", update_dtype=dtype, max_refine=20)
    dA = [T.colmajor(a) for a in As]
    dB = [T.colmajor(b) for b in Bs]
    work = T.lstsq_batched_workspace(shapes, 1, o)
    info = torch.full((len(shapes),), -7, dtype=torch.int32, device="cuda")
    Xs = T.lstsq_batched(dA, dB, o, work=work, info=info)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0] * len(shapes)
    X = [x.cpu().numpy()[:, 0] for x in Xs]
    for i, (A0, B0) in enumerate(zip(As, Bs)):
        assert H.ls_backward_error(A0, B0[:, 0], X[i]) <= 50 * EPS, (i, shapes[i])
    # x against the oracle's x on a sample: the largest member and every
    # eighth one.  Both solutions are exact for perturbations of relative
    # 2-norm size eta = 50 eps ||A||_F / ||A||_2, so by Wedin's least-squares
    # perturbation bound each lies within kappa eta (2 + (kappa + 1) ||r|| /
    # (||A||_2 ||x||)) ||x|| of the exact solution (the residual term
    # dominates for these random right-hand sides).
    sample = sorted({int(np.argmax([m * n for m, n in shapes]))} | set(range(0, len(shapes), 8)))
    for i in sample:
        xo, _, _ = H.lstsq(As[i], Bs[i][:, 0])
        a2 = np.linalg.norm(As[i], 2)
        kap = np.linalg.cond(As[i])
        eta = 50 * EPS * np.linalg.norm(As[i]) / a2
        r = np.linalg.norm(Bs[i][:, 0] - As[i] @ xo)
        bound = kap * eta * (2 + (kap + 1) * r / (a2 * np.linalg.norm(xo))) * np.linalg.norm(xo)
        assert np.linalg.norm(X[i] - xo) <= 2 * bound, (i, shapes[i])
