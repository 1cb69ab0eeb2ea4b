"""Helpers for the GPU parity tests: tolerances and oracle comparisons.

FP64 bar (the project's accuracy target): the factorization's normwise
backward error ||A - Q R||_F / ||A||_F <= 50 eps, eps = 2^-52.  Elementwise
comparison of R with the oracle's: both are backward stable to that bar, so
by first-order QR perturbation theory ||R_hat - D R_oracle||_F <=
2 sqrt(2) kappa_2(A) * 50 eps ||A||_F, D = diag(+-1) (R is unique up to
row signs for a full-rank A).  Q^T b restricted to its first n entries obeys
the same bound scaled by ||b||."""
import sys

import numpy as np

EPS = np.finfo(np.float64).eps


def case(msg):
    print("CASE", msg, flush=True)
    sys.stdout.flush()


def r_tol(A):
    return 2.0 * np.sqrt(2.0) * np.linalg.cond(A) * 50 * EPS * np.linalg.norm(A)
