"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import paper_1303_3182_amd as T
import synth
from oracle import householder as H
from tests.gpu_util import EPS, case, r_tol, trace_violations

pytestmark = pytest.mark.gpu


def _factor(A0, opts, nrhs=None):
    A = T.colmajor(A0)
    A, W = T.factor(A, opts, nrhs=A0.shape[1] if nrhs is None else nrhs)
    torch.cuda.synchronize()
    return A, W


def _check_factorization(A0, A, W, opts, tag):
    m, n = A0.shape
    Rg = np.triu(A.cpu().numpy()[:n, :n])
    Ro, Vo, tau = H.qr(A0)
    Ra, d = H.row_sign_align(Rg, Ro)
    err = np.linalg.norm(Ra - Ro)
    assert err <= r_tol(A0), (tag, "R vs oracle", err, r_tol(A0))
    # backward error through the library's own Q^T: ||Q^T A - [R; 0]||_F
    Bm = T.colmajor(A0)
    T.apply_qt(A, W, Bm, opts)
    torch.cuda.synchronize()
    QtA = Bm.cpu().numpy()
    QtA[:n] -= Rg
    be = np.linalg.norm(QtA) / np.linalg.norm(A0)
    assert be <= 50 * EPS, (tag, "backward error", be / EPS)
    return Rg, d


@pytest.mark.parametrize("nb,ib", [(32, 16), (64, 16), (64, 32), (128, 32), (256, 32)])
def test_single_tile_geqrt_matches_oracle(nb, ib):
    """p = q = 1: GEQRT alone is the oracle's Householder sequence, so R,
    the reflectors V and tau (the diagonal of T) match sign for sign."""
    for (m, n) in [(nb, nb), (nb - 7, nb - 9)]:
        case("geqrt nb=%d ib=%d m=%d n=%d" % (nb, ib, m, n))
        A0 = synth.gaussian(m, n, nb + m)
        o = T.default_opts(nb=nb, ib=ib)
        A, W = _factor(A0, o)
        out = A.cpu().numpy()
        Ro, Vo, tau = H.qr(A0)
        tol = r_tol(A0)
        assert np.linalg.norm(np.triu(out[:n, :n]) - Ro) <= tol
        assert np.linalg.norm(np.tril(out, -1) - np.tril(Vo, -1)) <= tol / np.linalg.norm(A0) * np.sqrt(n) * 10
        Tw = W.view(torch.float64)[32:32 + ib * nb].cpu().numpy().reshape(nb, ib)  # header is 256 bytes
        tdiag = np.array([Tw[c, c % ib] for c in range(n)])
        assert np.abs(tdiag - tau).max() <= 1e-12


SHAPES = [
    (512, 256, 128),   # 4 x 2 tiles (the smallest configuration)
    (300, 200, 64),    # ragged rows and columns
    (1000, 333, 64),   # 16 x 6, ragged
    (257, 257, 32),    # square, 1-row/1-col ragged tail
    (640, 640, 128),   # square 5 x 5
    (2048, 512, 256),  # 8 x 2 at nb 256
    (130, 3, 32),      # thin: one ragged tile column
]


@pytest.mark.parametrize("kernels", ["tt", "hybrid"])
@pytest.mark.parametrize("tree,param", [("flat", 0), ("binary", 0), ("fibonacci", 0), ("greedy", 0),
                                        ("grasap", 0), ("asap", 0), ("plasma", 3)])
def test_factor_matches_oracle(tree, param, kernels):
    for (m, n, nb) in SHAPES:
        case("factor %s(%d) %s m=%d n=%d nb=%d" % (tree, param, kernels, m, n, nb))
        A0 = synth.gaussian(m, n, m * 7 + n)
        o = T.default_opts(nb=nb, ib=16 if nb == 32 else 32, tree=tree, param=param, kernels=kernels)
        A, W = _factor(A0, o)
        _check_factorization(A0, A, W, o, (tree, kernels, m, n, nb))


@pytest.mark.parametrize("kernels", ["tt", "hybrid"])
def test_persistent_equals_sequential_bitwise(kernels):
    """The persistent executor and the one-launch-per-task reference run the
    same kernels on the same inputs in a dependency-respecting order, so the
    results are identical bit for bit."""
    for (m, n, nb) in [(512, 256, 128), (1000, 333, 64), (1536, 768, 256)]:
        case("bitwise %s m=%d n=%d nb=%d" % (kernels, m, n, nb))
        A0 = synth.gaussian(m, n, 5)
        outs = []
        for ex in (T.EXEC_PERSISTENT, T.EXEC_SEQUENTIAL):
            o = T.default_opts(nb=nb, tree="greedy", kernels=kernels, exec=ex)
            A, W = _factor(A0, o)
            outs.append((A.cpu().numpy(), W.cpu().numpy()))
        assert np.array_equal(outs[0][0], outs[1][0])


@pytest.mark.parametrize("tree,kernels", [("flat", "hybrid"), ("greedy", "tt"), ("plasma", "hybrid")])
def test_queue_orders_give_identical_results(tree, kernels):
    """The static list order changes only the order in which tasks start:
    the least-squares solution and the factors are identical bit for bit to
    those of the queue filled as tasks become ready, in both its orders."""
    for (m, n, nb) in [(1280, 1280, 128), (2000, 700, 64), (3072, 1024, 256)]:
        case("critical queue %s %s m=%d n=%d nb=%d" % (tree, kernels, m, n, nb))
        A0 = synth.gaussian(m, n, 21)
        b0 = synth.gaussian_rhs(m, 1, 21)
        outs = []
        for pr in ("static", "bottom", "list"):
            o = T.default_opts(nb=nb, tree=tree, param=2 if tree == "plasma" else 0, kernels=kernels,
                               priority=pr)
            X = T.lstsq(T.colmajor(A0), T.colmajor(b0), o)
            A, W = _factor(A0, o)
            outs.append((X.cpu().numpy(), A.cpu().numpy()))
        for x in outs[1:]:
            assert np.array_equal(outs[0][0], x[0]) and np.array_equal(outs[0][1], x[1])
        assert H.ls_backward_error(A0, b0[:, 0], outs[0][0][:, 0]) <= 50 * EPS


@pytest.mark.parametrize("stripes", [1, 2, 4, 8])
def test_stripes_do_not_change_results(stripes):
    case("stripes %d" % stripes)
    A0 = synth.gaussian(1024, 512, 9)
    o = T.default_opts(nb=256, tree="greedy", stripes=stripes)
    A, W = _factor(A0, o)
    _check_factorization(A0, A, W, o, ("stripes", stripes))


@pytest.mark.parametrize("kernels", ["tt", "hybrid"])
def test_apply_qt_and_lstsq(kernels):
    # nrhs <= 8 takes the one-wave-per-column back-substitution, larger
    # counts the blocked one
    for (m, n, nb, nrhs) in [(512, 256, 128, 1), (1000, 333, 64, 5), (700, 700, 128, 3), (4096, 300, 256, 2),
                             (600, 200, 64, 40), (300, 100, 32, 7), (520, 260, 256, 9)]:
        case("apply/lstsq %s m=%d n=%d nb=%d nrhs=%d" % (kernels, m, n, nb, nrhs))
        A0 = synth.gaussian(m, n, 11 + m)
        B0 = synth.gaussian_rhs(m, nrhs, 11 + m)
        o = T.default_opts(nb=nb, ib=16 if nb == 32 else 32, tree="grasap", kernels=kernels)
        A, W = _factor(A0, o)
        Bm = T.colmajor(B0)
        T.apply_qt(A, W, Bm, o)
        X = T.lstsq(T.colmajor(A0), T.colmajor(B0), o)
        torch.cuda.synchronize()
        Rg = np.triu(A.cpu().numpy()[:n, :n])
        Ro, Vo, tau = H.qr(A0)
        _, d = H.row_sign_align(Rg, Ro)
        QtB = Bm.cpu().numpy()
        QtBo = H.apply_qt(Vo, tau, B0)
        tol = r_tol(A0) / np.linalg.norm(A0)
        for c in range(nrhs):
            nb_ = np.linalg.norm(B0[:, c])
            assert np.linalg.norm(QtB[:n, c] * d - QtBo[:n, c]) <= tol * nb_
            assert abs(np.linalg.norm(QtB[n:, c]) - np.linalg.norm(QtBo[n:, c])) <= tol * nb_
            x = X.cpu().numpy()[:, c]
            assert H.ls_backward_error(A0, B0[:, c], x) <= 50 * EPS
            xo = H.back_substitute(Ro, QtBo[:n, c])
            kap = np.linalg.cond(A0)
            assert np.linalg.norm(x - xo) <= 100 * kap ** 2 * EPS * np.linalg.norm(xo) + 1e-300
        # the fused least-squares graph runs the same kernels in the same
        # per-tile order as factor + apply_qt + solve_r: identical bits
        T.solve_r(A, W, Bm, o)
        torch.cuda.synchronize()
        assert np.array_equal(Bm.cpu().numpy()[:n], X.cpu().numpy())


def test_edge_cases():
    for (m, n, nb) in [(1, 1, 32), (5, 1, 32), (33, 33, 32), (33, 1, 32), (64, 64, 64), (65, 64, 64), (200, 199, 64)]:
        case("edge m=%d n=%d nb=%d" % (m, n, nb))
        A0 = synth.gaussian(m, n, m + n)
        o = T.default_opts(nb=nb, ib=16, tree="greedy")
        A, W = _factor(A0, o)
        _check_factorization(A0, A, W, o, ("edge", m, n, nb))
    # upper-triangular input: every reflector is the identity (tau = 0), R = A
    case("edge triangular")
    A0 = np.asfortranarray(np.vstack([np.triu(synth.gaussian(96, 96, 1)), np.zeros((32, 96))]))
    A, W = _factor(A0, T.default_opts(nb=32, ib=16, tree="greedy"))
    assert np.array_equal(np.triu(A.cpu().numpy()[:96]), np.triu(A0[:96]))


def test_zero_column_reports_singular_r():
    case("singular lstsq")
    A0 = synth.gaussian(300, 100, 3)
    A0[:, 40] = 0.0
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    T.lstsq(T.colmajor(A0), T.colmajor(synth.gaussian_rhs(300, 1, 3)), T.default_opts(nb=64), info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == 41


def test_tall_skinny_full_size_five_trees():
    """16384 x 2048, nb = 256 (64 x 8 tiles), the five trees on identical
    inputs.  The oracle computes the first tile column's R and the first
    256 entries of Q^T b (they depend on A[:, :256] only); the whole R is
    checked through R^T R = A^T A on random probes, and |R(j,j)| must agree
    across trees."""
    m, n, nb = 16384, 2048, 256
    A0 = synth.gaussian(m, n, 1)
    b0 = synth.gaussian_rhs(m, 1, 1)
    Ro1, Vo1, tau1 = H.qr(A0[:, :nb])
    co1 = H.apply_qt(Vo1, tau1, b0[:, 0])[:nb]
    diags = []
    for tree in ["flat", "binary", "fibonacci", "greedy", "grasap"]:
        case("tall-skinny %s" % tree)
        o = T.default_opts(nb=nb, tree=tree)
        A, W = _factor(A0, o)
        Bm = T.colmajor(b0)
        T.apply_qt(A, W, Bm, o)
        torch.cuda.synchronize()
        R = np.triu(A[:n, :n].cpu().numpy())
        R1a, d1 = H.row_sign_align(R[:nb, :nb], Ro1)
        assert np.linalg.norm(R1a - Ro1) <= r_tol(A0[:, :nb])
        c = Bm[:nb, 0].cpu().numpy() * d1
        assert np.linalg.norm(c - co1) <= r_tol(A0[:, :nb]) / np.linalg.norm(A0[:, :nb]) * np.linalg.norm(b0)
        assert H.gram_error(A0, R) <= 50 * EPS
        assert abs(np.linalg.norm(Bm.cpu().numpy()) - np.linalg.norm(b0)) <= 50 * EPS * np.linalg.norm(b0)
        diags.append(np.abs(np.diag(R)))
    for dg in diags[1:]:
        assert np.max(np.abs(dg - diags[0]) / diags[0]) <= 1e-10


@pytest.mark.parametrize("kernels,priority", [("tt", "bottom"), ("hybrid", "bottom"), ("tt", "static"),
                                               ("hybrid", "static")])
def test_executor_trace_respects_dependencies(kernels, priority):
    """Post-hoc check of a normal run: with per-task clock stamps on, every
    task of the least-squares graph ran, and no task started before any of
    its predecessors had ended (the executor's data-flow contract), with one
    ready queue filled as tasks become ready and with the static list order."""
    for (m, n, nb, ib) in [(1000, 333, 64, 16), (2048, 768, 256, 32)]:
        case("trace %s %s m=%d n=%d nb=%d" % (kernels, priority, m, n, nb))
        o = T.default_opts(nb=nb, ib=ib, tree="greedy", kernels=kernels, priority=priority)
        nt = len(T.debug_graph(m, n, o, nrhs=1, kind=3))
        off, succ = T.debug_succ(m, n, o, nrhs=1, kind=3)
        buf = torch.zeros(4 * nt, dtype=torch.int64, device="cuda")
        A0 = synth.gaussian(m, n, 3)
        b0 = synth.gaussian_rhs(m, 1, 3)
        T.debug_trace(buf.data_ptr(), nt)
        try:
            X = T.lstsq(T.colmajor(A0), T.colmajor(b0), o)
            torch.cuda.synchronize()
        finally:
            T.debug_trace(None, 0)
        assert trace_violations(off, succ, buf.cpu().numpy(), nt) == []
        assert H.ls_backward_error(A0, b0[:, 0], X.cpu().numpy()[:, 0]) <= 50 * EPS


@pytest.mark.parametrize("priority", ["bottom", "static"])
def test_watchdog_fires_and_the_executor_drains(priority):
    """Failure handling forced from the host: with a watchdog limit of one
    clock tick, a workgroup that finds its queue slot not yet filled aborts
    the launch; every workgroup then leaves, info reports the timeout, and
    the next launch (default limit) is correct again."""
    case("watchdog %s" % priority)
    A0 = synth.gaussian(512, 256, 4)
    o = T.default_opts(nb=128, tree="flat", kernels="hybrid", priority=priority)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    T.debug_spin_limit(1)
    try:
        T.factor(T.colmajor(A0), o, info=info)
        torch.cuda.synchronize()
    finally:
        T.debug_spin_limit(0)
    assert int(info.item()) == -1000  # TQR_INFO_TIMEOUT
    A, W = _factor(A0, o)
    _check_factorization(A0, A, W, o, "after watchdog")


@pytest.mark.parametrize("s", [530, -530])
@pytest.mark.parametrize("kernels", ["tt", "hybrid"])
def test_extreme_scaling(s, kernels):
    """Entries near the FP64 overflow (2^530 ~ 1e160) or underflow (2^-530)
    threshold, where the unscaled squares of a Householder norm over- or
    underflow: R equals 2^s times the oracle's R of the unscaled matrix (to
    the FP64 bar) and the least-squares solution meets 50 eps."""
    for (m, n, nb) in [(700, 300, 64), (1024, 512, 256)]:
        case("scaling 2^%d %s m=%d n=%d nb=%d" % (s, kernels, m, n, nb))
        A0 = synth.gaussian(m, n, 40 + m)
        b0 = synth.gaussian_rhs(m, 1, 40 + m)
        As, bs = A0 * 2.0 ** s, b0 * 2.0 ** s
        o = T.default_opts(nb=nb, tree="greedy", kernels=kernels)
        A, W = _factor(As, o)
        R = np.triu(A.cpu().numpy()[:n, :n]) * 2.0 ** -s
        Ro, _, _ = H.qr(A0)
        Ra, _ = H.row_sign_align(R, Ro)
        assert np.all(np.isfinite(R))
        assert np.linalg.norm(Ra - Ro) <= r_tol(A0)
        X = T.lstsq(T.colmajor(As), T.colmajor(bs), o)
        torch.cuda.synchronize()
        assert H.ls_backward_error(As, bs[:, 0], X.cpu().numpy()[:, 0]) <= 50 * EPS


def test_tiny_subdiagonal_is_still_reduced():
    """A column whose entries below the diagonal are far below the
    underflow threshold of their squares (1e-170 under a unit diagonal)
    still gets a reflector that zeroes them (tau = 0 only for an exactly
    zero column), as in the oracle."""
    case("tiny subdiagonal")
    A0 = np.asfortranarray(np.vstack([np.eye(64), 1e-170 * synth.gaussian(64, 64, 5)]))
    o = T.default_opts(nb=64, ib=16, tree="greedy")
    A, W = _factor(A0, o)
    R = np.triu(A.cpu().numpy()[:64, :64])
    Ro, _, _ = H.qr(A0)
    assert np.array_equal(np.sign(np.diag(R)), np.sign(np.diag(Ro)))
    Bm = T.colmajor(A0)
    T.apply_qt(A, W, Bm, o)
    torch.cuda.synchronize()
    assert np.abs(Bm.cpu().numpy()[64:]).max() <= 1e-10 * 1e-170
