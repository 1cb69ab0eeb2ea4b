"""Pins of the selector network's oracle (oracle/mlp.py) to things other
than itself: central finite differences of its own plain forward pass,
closed forms of degenerate networks, and Adam's first step."""
import numpy as np

from oracle import mlp as M


def _rand(seed, B=7):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(M.P) * 0.3
    X = rng.standard_normal((B, M.F))
    t = rng.standard_normal(B)
    return w, X, t


def _fd_check(grad_fn, seed):
    w, X, t = _rand(seed)
    g = grad_fn(w, X, t)
    rng = np.random.default_rng(seed + 100)
    idx = rng.choice(M.P, 60, replace=False)
    h = 1e-6
    worst = 0.0
    for p in idx:
        e = np.zeros(M.P)
        e[p] = h
        fd = (M.loss(w + e, X, t) - M.loss(w - e, X, t)) / (2 * h)
        worst = max(worst, abs(fd - g[p]) / (abs(fd) + 1e-8))
    return worst


def test_gradient_matches_finite_differences():
    for seed in range(3):
        assert _fd_check(M.grad, seed) <= 1e-5


def test_planted_mistake_in_gradient_is_caught():
    """Dropping the tanh derivative of the second hidden layer (a plausible
    slip) makes the finite-difference pin fail."""
    def bad_grad(w, X, t):
        W1, b1, W2, b2, W3, b3 = M.unpack(w)
        B = X.shape[0]
        h1 = np.tanh(X @ W1.T + b1)
        h2 = np.tanh(h1 @ W2.T + b2)
        dy = 2.0 * (h2 @ W3 + b3 - t) / B
        dz2 = np.outer(dy, W3)                      # missing (1 - h2^2)
        dz1 = (dz2 @ W2) * (1.0 - h1 ** 2)
        return M.pack(dz1.T @ X, dz1.sum(0), dz2.T @ h1, dz2.sum(0), h2.T @ dy, dy.sum())
    assert _fd_check(bad_grad, 0) > 1e-2


def test_degenerate_networks_closed_forms():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((4, M.F))
    z = np.zeros(M.P)
    z[-1] = 1.25                                    # only b3
    assert np.allclose(M.forward(z, X), 1.25)
    W1, b1, W2, b2, W3, b3 = M.unpack(rng.standard_normal(M.P))
    W1[:] = 0.0
    W2[:] = 0.0
    w = M.pack(W1, b1, W2, b2, W3, b3)
    assert np.allclose(M.forward(w, X), W3 @ np.tanh(b2) + b3)
    # a perfect prediction has zero loss and zero gradient
    t = M.forward(w, X)
    assert M.loss(w, X, t) == 0.0 and np.all(M.grad(w, X, t) == 0.0)
    # one hidden-1 unit, linear regime: d y / d b3 = 1 for every sample, so
    # the b3 gradient is 2 mean(y - t)
    w2, X2, t2 = _rand(9)
    g = M.grad(w2, X2, t2)
    assert np.isclose(g[-1], 2.0 * np.mean(M.forward(w2, X2) - t2))


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    w = rng.standard_normal(M.P)
    g = rng.standard_normal(M.P)
    w1, m1, m2 = M.adam_step(w, g, np.zeros(M.P), np.zeros(M.P), 1, 0.01)
    # bias-corrected moments equal g and g^2 after one step
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)
