#!/usr/bin/env python3
"""Benchmark of the tiled QR path on one MI355X.

Workload: FP64 least squares on a tall-skinny matrix, m = 16384, n = 2048,
tile nb = 256 (64 x 8 tiles), entries i.i.d. N(0,1) (seeded, synthetic),
GrASAP elimination tree, TT kernels.  One step is the whole hot path on one
batch: tqr_lstsq, i.e. copy A and b into the workspace, then one persistent
executor launch that factors A = QR, applies Q^T to b as the factorization
proceeds, and back-substitutes R x = (Q^T b)(1:n) (elimination list and
task graph are cached after the first call).

value = 2 n^2 (m - n/3) / (seconds per step), in TFLOP/s: only the QR flops
are counted although the step also applies Q^T and solves.  Inputs are
resident in HBM when the timed region starts.

The JSON line also carries the roofline of the dominant kernel (the
executor launch, timed by HIP events that the library records around each
launch on the launch's stream, inside the timed region) and the CPU oracle
timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QR TFLOP/s (2n²(m−n/3)) plain FP64 vs mixed+refined at equal FP64 error"
PEAK_FP64_MFMA = 78.6  # TFLOP/s, MI355X dense FP64 matrix peak


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def qr_flops(m, n):
    return 2.0 * n * n * (m - n / 3.0)


def cpu_baseline(A0, ncols):
    """The FP64 oracle (unblocked Householder, numpy) on the first `ncols`
    columns of the workload matrix: a bounded sample, rate in TFLOP/s of the
    same flop formula."""
    from oracle import householder as H
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        cores = 1
    S = A0[:, :ncols].copy(order="F")
    t0 = time.perf_counter()
    H.qr(S)
    dt = time.perf_counter() - t0
    m = S.shape[0]
    return {"value": qr_flops(m, ncols) / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores),
            "kind": "oracle", "seconds": dt,
            "sample": "unblocked FP64 Householder QR of the first %d columns of the %dx%d workload "
                      "matrix (%d x %d)" % (ncols, m, A0.shape[1], m, ncols)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--m", type=int, default=16384)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--ib", type=int, default=32)
    ap.add_argument("--tree", default="grasap")
    ap.add_argument("--kernels", default="tt")
    ap.add_argument("--stripes", type=int, default=0)
    ap.add_argument("--cpu-sample-cols", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed", nargs="*", default=["f32", "bf16"],
                    help="also time the solve with these update dtypes + FP64 refinement")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the factorization runs on a single device "
              "and there is no multi-GPU path; use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1303_3182_amd as T
    import synth

    m, n, nb = args.m, args.n, args.nb
    log("workload %dx%d nb=%d tree=%s kernels=%s" % (m, n, nb, args.tree, args.kernels))
    A0 = synth.gaussian(m, n, 1)
    b0 = synth.gaussian_rhs(m, 1, 1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    opts = T.default_opts(nb=nb, ib=args.ib, tree=args.tree, kernels=args.kernels, stripes=args.stripes)
    A = T.colmajor(A0, dev)
    b = T.colmajor(b0, dev)
    X = torch.empty((1, n), dtype=torch.float64, device=dev).t()
    work = T.lstsq_workspace(m, n, 1, opts, dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)

    def step():
        T.lstsq(A, b, opts, X=X, work=work, info=info)

    for w in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done (%d steps)" % args.warmup)
    T.debug_timing(True)
    t0 = time.perf_counter()
    for s in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, launches = T.debug_timing_read()
    T.debug_timing(False)
    ms = (t1 - t0) / args.steps * 1e3
    factor_ms = kern_ms / launches
    log("timed %d steps: %.3f ms/step, executor launch %.3f ms (%d launches)" % (args.steps, ms, factor_ms, launches))
    if int(info.item()) != 0:
        raise SystemExit("executor reported info=%d" % int(info.item()))

    # accuracy of the last step's solution: Stewart's one-sided backward
    # error bound ||A^T r|| / (||A||_F ||r||) in extended precision
    Al = A0.astype(np.longdouble)

    def backward_error(x):
        r = b0[:, 0].astype(np.longdouble) - Al @ x.astype(np.longdouble)
        return float(np.linalg.norm((Al.T @ r).astype(np.float64)) /
                     (np.linalg.norm(A0) * np.linalg.norm(r.astype(np.float64))))

    be = backward_error(X[:, 0].cpu().numpy())

    # the same least-squares solve with low-precision trailing updates and
    # FP64 refinement to the FP64 backward error
    mixed = {}
    for dt in args.mixed:
        om = T.default_opts(nb=nb, ib=args.ib, tree=args.tree, kernels=args.kernels, stripes=args.stripes,
                            update_dtype=dt, max_refine=20)
        wm = T.lstsq_workspace(m, n, 1, om, dev)
        for w in range(args.warmup):
            T.lstsq(A, b, om, X=X, work=wm, info=info)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.steps):
            T.lstsq(A, b, om, X=X, work=wm, info=info)
        torch.cuda.synchronize()
        mms = (time.perf_counter() - t0) / args.steps * 1e3
        rep = T.refine_report(wm)
        inf = int(info.item())
        mbe = backward_error(X[:, 0].cpu().numpy())
        log("mixed %s: %.3f ms/step, %d refinement steps, backward error %.2e (info %d)" %
            (dt, mms, rep["iterations"], mbe, inf))
        mixed[dt] = {"ms_per_step": mms, "value": qr_flops(m, n) / (mms / 1e3) / 1e12, "unit": "TFLOP/s",
                     "speedup_vs_fp64": ms / mms, "refine_steps": rep["iterations"], "converged": rep["done"],
                     "info": inf, "ls_backward_error": mbe, "equal_fp64_error": bool(mbe <= 50 * 2.0 ** -52)}

    flops = qr_flops(m, n)
    achieved = flops / (factor_ms / 1e3) / 1e12
    out = {
        "metric": METRIC,
        "value": flops / (ms / 1e3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FP64 tiled-QR least squares, tall-skinny %dx%d, nb=%d (%dx%d tiles), "
                               "N(0,1) entries, seed 1" % (m, n, nb, -(-m // nb), -(-n // nb)),
                   "m": m, "n": n, "nb": nb, "ib": args.ib, "tree": args.tree,
                   "kernels": args.kernels, "precision": "plain FP64"},
        "executor_ms": factor_ms,
        "ls_backward_error": be,
        "mixed_precision": mixed,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_MFMA, "traffic": None,
                     "kernel": "exec_persistent (least-squares task graph: factor, Q^T b, R x = c)"},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a %d-column sample" % args.cpu_sample_cols)
        out["cpu_baseline"] = cpu_baseline(A0, args.cpu_sample_cols)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
