"""Oracle of the selector network (test infrastructure only): forward pass,
mean-squared-error loss, its gradient by the chain rule, and one Adam step,
in FP64 numpy, written from the definitions.

Network: y = W3 . tanh(W2 tanh(W1 x + b1) + b2) + b3, with the parameter
vector laid out as W1 [H x F] row-major, b1 [H], W2 [H x H] row-major
(W2[j, k] maps hidden-1 unit k to hidden-2 unit j), b2 [H], W3 [H], b3.
Loss over a batch: mean((y - t)^2).  Adam: Kingma and Ba, "Adam: a method
for stochastic optimization", ICLR 2015, algorithm 1 (beta1 0.9, beta2
0.999, eps 1e-8).  (The selector is a project addition; the thesis has no
learned component.)
"""
import numpy as np

H = 64
F = 9
P = H * F + H + H * H + H + H + 1


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (P,)
    o = 0
    W1 = w[o:o + H * F].reshape(H, F)
    o += H * F
    b1 = w[o:o + H]
    o += H
    W2 = w[o:o + H * H].reshape(H, H)
    o += H * H
    b2 = w[o:o + H]
    o += H
    W3 = w[o:o + H]
    o += H
    b3 = w[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, [b3]])


def forward(w, X):
    """Predictions for the rows of X (batch x F)."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ W3 + b3


def loss(w, X, t):
    return float(np.mean((forward(w, X) - np.asarray(t, dtype=np.float64)) ** 2))


def grad(w, X, t):
    """Gradient of loss(w, X, t) with respect to w, by the chain rule."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    B = X.shape[0]
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = h2 @ W3 + b3
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / B      # dL/dy, per sample
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    dz2 = np.outer(dy, W3) * (1.0 - h2 ** 2)                  # B x H
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - h1 ** 2)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(w, g, m1, m2, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step from moments (m1, m2) at step t >= 1; returns the new
    (w, m1, m2)."""
    m1 = b1 * m1 + (1.0 - b1) * g
    m2 = b2 * m2 + (1.0 - b2) * g * g
    mh = m1 / (1.0 - b1 ** t)
    vh = m2 / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m1, m2
