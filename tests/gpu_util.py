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


def trace_violations(off, succ, trace, ntasks, slack=0):
    """Post-hoc dependency check of an executor trace (host only).

    off/succ: the task graph's successor lists (CSR); trace: int64 array of
    4 entries per task {start, end, workgroup, cu} in device wall-clock
    ticks.  Every task must have run (end >= start > 0) and every successor
    must start no earlier than its predecessor ended (minus `slack` ticks).
    Returns the list of violations (empty when the trace is consistent)."""
    tr = np.asarray(trace, dtype=np.int64).reshape(-1, 4)
    bad = []
    for t in range(ntasks):
        if not (tr[t, 0] > 0 and tr[t, 1] >= tr[t, 0]):
            bad.append(("not run", t))
    for t in range(ntasks):
        for e in range(off[t], off[t + 1]):
            s = succ[e]
            if tr[s, 0] + slack < tr[t, 1]:
                bad.append(("order", t, s, int(tr[t, 1] - tr[s, 0])))
    return bad
