"""Batched ragged least squares (one executor launch for the whole batch)
and the batch autotuner, through the C ABI, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import paper_1303_3182_amd as T
import synth
from oracle import householder as H
from tests.gpu_util import EPS, case

pytestmark = pytest.mark.gpu


def _batch(count, seed, m_range, n_range, nrhs=1):
    shapes = synth.ragged_batch_shapes(count, seed, m_range, n_range)
    As, Bs = synth.ragged_batch(shapes, seed, nrhs)
    return shapes, As, Bs


def _check(shapes, As, Bs, Xs, tag):
    for x, ((m, n), A0, B0) in enumerate(zip(shapes, As, Bs)):
        X = Xs[x].cpu().numpy()
        for c in range(B0.shape[1]):
            be = H.ls_backward_error(A0, B0[:, c], X[:, c])
            assert be <= 50 * EPS, (tag, x, m, n, be / EPS)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nb,ib,tree", [(64, 16, "auto"), (128, 32, "greedy"), (32, 16, "flat")])
def test_batched_matches_oracle(dtype, nb, ib, tree):
    shapes, As, Bs = _batch(24, 3, (40, 1500), (3, 300))
    case("batched %s nb=%d tree=%s shapes=%s" % (dtype, nb, tree, shapes[:4]))
    o = T.default_opts(nb=nb, ib=ib, tree=tree, update_dtype=dtype, max_refine=20)
    dA = [T.colmajor(a) for a in As]
    dB = [T.colmajor(b) for b in Bs]
    work = T.lstsq_batched_workspace(shapes, 1, o)
    info = torch.full((len(shapes),), -7, dtype=torch.int32, device="cuda")
    Xs = T.lstsq_batched(dA, dB, o, work=work, info=info)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0] * len(shapes)
    _check(shapes, As, Bs, Xs, (dtype, nb, tree))
    reps = T.refine_reports(work, len(shapes))
    if dtype == "f64":
        assert all(r["done"] == 0 and r["iterations"] == 0 for r in reps)
    else:
        assert all(r["done"] == 1 for r in reps)
        assert max(r["iterations"] for r in reps) >= 1


def test_batched_equals_single_problem_solves():
    """In FP64 each problem of the batch runs exactly the kernels of a
    single-problem lstsq on the same tile graph: identical bits."""
    shapes, As, Bs = _batch(9, 5, (100, 900), (10, 200), nrhs=2)
    o = T.default_opts(nb=64, ib=16, tree="greedy")
    dA = [T.colmajor(a) for a in As]
    dB = [T.colmajor(b) for b in Bs]
    Xs = T.lstsq_batched(dA, dB, o)
    torch.cuda.synchronize()
    for x in range(len(shapes)):
        Xi = T.lstsq(dA[x], dB[x], o)
        torch.cuda.synchronize()
        assert np.array_equal(Xi.cpu().numpy(), Xs[x].cpu().numpy()), x


def test_batched_rank_deficient_member_reports_only_itself():
    shapes, As, Bs = _batch(6, 9, (100, 600), (10, 90))
    As[2][:, 3] = 0.0
    dA = [T.colmajor(a) for a in As]
    dB = [T.colmajor(b) for b in Bs]
    info = torch.zeros(len(shapes), dtype=torch.int32, device="cuda")
    T.lstsq_batched(dA, dB, T.default_opts(nb=64, ib=16), info=info)
    torch.cuda.synchronize()
    got = info.cpu().tolist()
    assert got[2] == 4 and all(v == 0 for i, v in enumerate(got) if i != 2), got


def test_autotuner_picks_a_built_config_and_caches():
    shapes, As, Bs = _batch(32, 11, (256, 2048), (32, 256))
    dA = [T.colmajor(a) for a in As]
    dB = [T.colmajor(b) for b in Bs]
    o = T.default_opts(tree="auto", update_dtype="f32")
    ms = T.autotune_batched(dA, dB, o)
    assert ms > 0 and (o.nb, o.ib) in [(32, 16), (64, 16), (64, 32), (128, 32), (256, 32)]
    assert T.autotune_batched(dA, dB, o) == -1.0   # cached
    Xs = T.lstsq_batched(dA, dB, o)
    torch.cuda.synchronize()
    _check(shapes, As, Bs, Xs, "autotuned")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batched_square_member_converges(dtype):
    """A square member of a low-precision batch is stopped by the
    Rigal-Gaches measure (its residual reaches rounding level), so it
    converges like the rectangular members instead of running out of
    refinement steps.  Classical refinement with BF16 factors contracts only
    when kappa * u_bf16 is well below one (u_bf16 = 2^-8), so the BF16
    case takes a square member of condition number 10 (a 200 x 200
    Gaussian matrix has kappa of order 1e3)."""
    shapes = [(300, 100), (200, 200), (500, 60)]
    As = [synth.gaussian(m, n, 70 + i) for i, (m, n) in enumerate(shapes)]
    if dtype == "bf16":
        As[1] = synth.conditioned(200, 10.0, 71)[0]
    Bs = [synth.gaussian_rhs(m, 1, 70 + i) for i, (m, n) in enumerate(shapes)]
    case("batched square member %s" % dtype)
    o = T.default_opts(nb=64, ib=16, tree="greedy", update_dtype=dtype, max_refine=20)
    dA = [T.colmajor(a) for a in As]
    dB = [T.colmajor(b) for b in Bs]
    work = T.lstsq_batched_workspace(shapes, 1, o)
    info = torch.full((len(shapes),), -7, dtype=torch.int32, device="cuda")
    Xs = T.lstsq_batched(dA, dB, o, work=work, info=info)
    torch.cuda.synchronize()
    reps = T.refine_reports(work, len(shapes))
    assert info.cpu().tolist() == [0] * len(shapes), reps
    assert all(r["done"] == 1 for r in reps), reps
    _check(shapes, As, Bs, Xs, ("square member", dtype))
