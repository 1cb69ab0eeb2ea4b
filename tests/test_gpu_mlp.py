"""The selector network's HIP kernels (forward, gradient, Adam, fitting)
against the FP64 oracle, and the selector wired into TQR_AUTO."""
import os

import numpy as np
import pytest
import torch

import paper_1303_3182_amd as T
from paper_1303_3182_amd import selector as S
import synth
from oracle import householder as H
from oracle import mlp as M
from tests.gpu_util import EPS, case

pytestmark = pytest.mark.gpu


def _data(seed, B):
    rng = np.random.default_rng(seed)
    w = (rng.standard_normal(M.P) * 0.2).astype(np.float32)
    X = rng.standard_normal((B, M.F)).astype(np.float32)
    t = rng.standard_normal(B).astype(np.float32)
    return w, X, t


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_forward_matches_oracle():
    for B in (1, 5, 300):
        case("mlp forward B=%d" % B)
        w, X, _ = _data(B, B)
        y = S.forward(_dev(w), _dev(X)).cpu().numpy()
        yo = M.forward(w.astype(np.float64), X.astype(np.float64))
        # FP32 arithmetic: a few hundred roundings of order 2^-24 each
        assert np.max(np.abs(y - yo)) <= 1e-4 * (1 + np.max(np.abs(yo)))


def test_gradient_matches_oracle():
    for B in (1, 64, 257):
        case("mlp grad B=%d" % B)
        w, X, t = _data(10 + B, B)
        g, loss = S.grad(_dev(w), _dev(X), _dev(t))
        go = M.grad(w.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
        lo = M.loss(w.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
        assert abs(float(loss.item()) - lo) <= 1e-4 * lo
        g = g.cpu().numpy()
        assert np.max(np.abs(g - go)) <= 1e-4 * np.max(np.abs(go))


def test_adam_step_matches_oracle():
    rng = np.random.default_rng(4)
    w = rng.standard_normal(M.P).astype(np.float32)
    g = rng.standard_normal(M.P).astype(np.float32)
    m1 = (rng.standard_normal(M.P) * 0.1).astype(np.float32)
    m2 = (rng.random(M.P) * 0.1).astype(np.float32)
    dw, dm1, dm2 = _dev(w), _dev(m1), _dev(m2)
    S.adam(dw, _dev(g), dm1, dm2, 3, 0.01)
    wo, m1o, m2o = M.adam_step(w.astype(np.float64), g.astype(np.float64), m1.astype(np.float64),
                               m2.astype(np.float64), 3, 0.01)
    assert np.allclose(dw.cpu().numpy(), wo, rtol=1e-5, atol=1e-6)
    assert np.allclose(dm1.cpu().numpy(), m1o, rtol=1e-5, atol=1e-7)
    assert np.allclose(dm2.cpu().numpy(), m2o, rtol=1e-5, atol=1e-8)


def test_fit_learns_a_teacher_network():
    """Targets from a random teacher network (the oracle's forward): the
    GPU fitting loop drives the loss down by two orders of magnitude."""
    rng = np.random.default_rng(8)
    teacher = rng.standard_normal(M.P) * 0.3
    X = rng.standard_normal((512, M.F))
    t = M.forward(teacher, X)
    p = S.init_params(1)
    hist = S.fit(p, _dev(X.astype(np.float32)), _dev(t.astype(np.float32)), 1500, 3e-3).cpu().numpy()
    assert hist[-1] <= 1e-2 * hist[0], (hist[0], hist[-1])
    final = M.loss(p.cpu().numpy().astype(np.float64), X, t)
    assert final <= 1e-2 * hist[0]


def test_auto_without_network_is_grasap_256_and_with_one_a_candidate():
    S.set_selector(None)
    assert S.select(5000, 300) == (T.GRASAP, 256, 32)
    p = S.init_params(7)
    S.set_selector(p)
    tree, nb, ib = S.select(5000, 300)
    assert tree in (T.FLAT, T.BINARY, T.FIBONACCI, T.GREEDY, T.GRASAP) and nb in (64, 128, 256)
    # the pick is the candidate with the smallest prediction (oracle forward)
    w = p.cpu().numpy().astype(np.float64)
    cands = [(t, b) for b in (64, 128, 256) for t in ("flat", "binary", "fibonacci", "greedy", "grasap")]
    preds = [M.forward(w, S.features(5000, 300, b, t)[None, :].astype(np.float64))[0] for t, b in cands]
    bt, bnb = cands[int(np.argmin(preds))]
    assert (T.TREES[bt], bnb) == (tree, nb)
    # TQR_AUTO through lstsq solves to the FP64 bar with that choice
    A0 = synth.gaussian(700, 300, 3)
    b0 = synth.gaussian_rhs(700, 1, 3)
    X = T.lstsq(T.colmajor(A0), T.colmajor(b0), T.default_opts(tree="auto"))
    torch.cuda.synchronize()
    assert H.ls_backward_error(A0, b0[:, 0], X.cpu().numpy()[:, 0]) <= 50 * EPS
    S.set_selector(None)


@pytest.mark.skipif(not os.path.exists(S.WEIGHTS), reason="no trained selector weights shipped")
def test_trained_selector_gain_over_fallback():
    """The shipped network (trained on engine timings) against GrASAP at
    nb = 256 on shapes it was not trained on: the total measured time of its
    picks is below the fallback's (the ratio is reported)."""
    p = S.load_selector()
    shapes = S.random_shapes(8, 99, max_elems=1 << 25)
    pick_ms = fall_ms = 0.0
    for i, (m, n) in enumerate(shapes):
        tid, nb, ib = S.select(m, n)
        tree = [t for t in S.TREES if T.TREES[t] == tid][0]
        a = S.time_factor(m, n, nb, tree, reps=3, seed=500 + i)
        f = S.time_factor(m, n, 256, "grasap", reps=3, seed=500 + i)
        case("selector %dx%d: pick %s nb=%d %.2f ms, fallback %.2f ms" % (m, n, tree, nb, a, f))
        pick_ms += a
        fall_ms += f
    print("selector gain over GrASAP@256 on %d held-out shapes: %.3fx" % (len(shapes), fall_ms / pick_ms))
    S.set_selector(None)
    assert pick_ms < fall_ms
    assert p is not None
