#!/usr/bin/env python3
"""Benchmark of the tiled QR path on one MI355X.

Default workload (--workload square): least squares on square 8192 x 8192
systems with prescribed condition number kappa in {1e2, 1e5, 1e8}:
A = U diag(sigma) V^T with Haar U, V and sigma_i = kappa^(-(i-1)/(n-1)),
b = A x + 1e-6 N(0,1) (seeded, synthetic).  Tile nb = 256 (32 x 32 tiles),
ib = 32, Greedy elimination tree, TT kernels.  One step is the whole hot
path on one system: tqr_lstsq, i.e. copy A and b into the workspace, then
one persistent executor launch that factors A = QR, applies Q^T to b as the
factorization proceeds and back-substitutes R x = (Q^T b)(1:n).  The value
is the plain FP64 solve; the same systems are then solved with FP32 and
BF16 trailing updates plus FP64 refinement to the FP64 backward error, per
kappa, and their speed-ups over FP64 (and any cell that did not reach the
FP64 error) are reported beside it.

Also in the JSON line:
  roofline    the dominant kernel (the executor launch) against the FP64
              matrix peak: QR flops / mean launch duration (HIP events the
              library records around each launch on the launch's stream);
  gamma_ub    the thesis's upper-bound model gamma_task T / max(T/P, cp)
              (section "Experimental results"), with the measured per-task
              rates of one traced launch;
  c2_trees    16384 x 2048 (64 x 8 tiles) FP64 least squares with the five
              trees of the thesis on identical inputs;
  cpu_baseline the FP64 oracle on a bounded column sample of the same matrix,
              single-threaded and with all host cores.

Other workloads (each prints its own JSON line):
  --workload tall     16384 x 2048 least squares (the five trees, mixed
                      precision, selector and a small tuning grid).
  --workload batched  512 ragged least-squares problems, m log-uniform in
                      [256, 8192], n log-uniform in [32, 512], n <= m/2,
                      N(0,1); FP32 updates + FP64 refinement, nb/ib from the
                      autotuner, tree per problem by critical path.

value = sum of 2 n^2 (m - n/3) over the problems / (seconds per step), in
TFLOP/s: only the QR flops are counted although the step also applies Q^T
and solves (and refines).  Inputs are resident in HBM when the timed region
starts.
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
EPS = 2.0 ** -52


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def qr_flops(m, n):
    return 2.0 * n * n * (m - n / 3.0)


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        return 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_qr_rate(S, what):
    """The FP64 oracle (unblocked Householder, numpy) on the sample S, as a
    rate in TFLOP/s of the same flop formula: once with every host core
    available to its BLAS calls and once single-threaded."""
    from threadpoolctl import threadpool_limits
    from oracle import householder as H
    m, n = S.shape
    runs = {}
    for label, threads in (("all_cores", None), ("single_thread", 1)):
        with threadpool_limits(limits=threads):
            cores = int(blas_threads())
            t0 = time.perf_counter()
            H.qr(S)
            dt = time.perf_counter() - t0
        runs[label] = {"value": qr_flops(m, n) / dt / 1e12, "seconds": dt, "cores": cores}
    out = {"value": runs["all_cores"]["value"], "unit": "TFLOP/s", "cores": runs["all_cores"]["cores"],
           "kind": "oracle", "seconds": runs["all_cores"]["seconds"], "sample": what,
           "single_thread": runs["single_thread"], "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    return out


def timed(fn, steps, warmup, torch, T):
    """Runs fn warmup times, then `steps` times inside the timed region;
    returns (ms per step by the host clock, mean executor launch ms, launches
    per step)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    T.debug_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, launches = T.debug_timing_read()
    T.debug_timing(False)
    return (t1 - t0) / steps * 1e3, kern_ms / max(launches, 1), launches / steps


def cold_cache_timing(np, torch, T, run_once, steps, flush_bytes=1 << 30):
    """Executor launch time after the caches beyond the CUs have been
    flushed: before each call a device buffer of flush_bytes (four times the
    256 MB Infinity Cache, and far larger than the L2s) is overwritten and
    the device synchronised; the call's executor launch is then timed with
    the library's HIP events, as in timed().  (The call's own copy of A into
    its workspace still runs first and leaves its tail cached.)"""
    buf = torch.empty(flush_bytes // 4, dtype=torch.int32, device="cuda")
    ms = []
    for _ in range(steps):
        buf.fill_(1)
        torch.cuda.synchronize()
        T.debug_timing(True)
        run_once()
        torch.cuda.synchronize()
        k, nl = T.debug_timing_read()
        T.debug_timing(False)
        ms.append(k / max(nl, 1))
    del buf
    return {"executor_ms": float(np.median(ms)), "executor_ms_all": ms, "flush_bytes": flush_bytes}


def recorded_traffic(record, workload):
    """HBM bytes per executor launch from a committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE measurement (profiles/traffic_*.json), or None when the
    sources of the measured kernel have changed since (their SHA-256 is
    recorded with the counts)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", record)
    try:
        with open(path) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        same = h.hexdigest() == rec["sha256"] and rec["workload"] == workload
        return rec["bytes_total"] if same else None
    except (OSError, KeyError, ValueError):
        return None


def roofline(flops, kernel_ms, kernel, traffic=None):
    achieved = flops / (kernel_ms / 1e3) / 1e12
    return {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_MFMA, "traffic": traffic, "kernel": kernel}


def base_line(args, value, ms, dtype, config):
    return {"metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


# --------------------------------------------------------------- tall-skinny
def run_tall(args, np, torch, T, synth):
    m, n, nb = args.m, args.n, args.nb
    log("workload %dx%d nb=%d tree=%s kernels=%s" % (m, n, nb, args.tree, args.kernels))
    A0 = synth.gaussian(m, n, 1)
    b0 = synth.gaussian_rhs(m, 1, 1)
    dev = torch.device("cuda:0")
    opts = T.default_opts(nb=nb, ib=args.ib, tree=args.tree, kernels=args.kernels, stripes=args.stripes)
    A = T.colmajor(A0, dev)
    b = T.colmajor(b0, dev)
    X = torch.empty((1, n), dtype=torch.float64, device=dev).t()
    work = T.lstsq_workspace(m, n, 1, opts, dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    ms, kms, _ = timed(lambda: T.lstsq(A, b, opts, X=X, work=work, info=info), args.steps, args.warmup, torch, T)
    log("timed %d steps: %.3f ms/step, executor launch %.3f ms" % (args.steps, ms, kms))
    if int(info.item()) != 0:
        raise SystemExit("executor reported info=%d" % int(info.item()))

    # accuracy: Stewart's one-sided backward error bound ||A^T r|| / (||A||_F ||r||)
    # in extended precision
    Al = A0.astype(np.longdouble)

    def backward_error(x):
        r = b0[:, 0].astype(np.longdouble) - Al @ x.astype(np.longdouble)
        return float(np.linalg.norm((Al.T @ r).astype(np.float64)) /
                     (np.linalg.norm(A0) * np.linalg.norm(r.astype(np.float64))))

    be = backward_error(X[:, 0].cpu().numpy())
    mixed = {}
    for dt in args.mixed:
        om = T.default_opts(nb=nb, ib=args.ib, tree=args.tree, kernels=args.kernels, stripes=args.stripes,
                            update_dtype=dt, max_refine=20)
        wm = T.lstsq_workspace(m, n, 1, om, dev)
        mms, mkms, nl = timed(lambda: T.lstsq(A, b, om, X=X, work=wm, info=info), args.steps, args.warmup,
                              torch, T)
        rep = T.refine_report(wm)
        inf = int(info.item())
        mbe = backward_error(X[:, 0].cpu().numpy())
        log("mixed %s: %.3f ms/step, %d refinement steps, backward error %.2e (info %d)" %
            (dt, mms, rep["iterations"], mbe, inf))
        mixed[dt] = {"ms_per_step": mms, "value": qr_flops(m, n) / (mms / 1e3) / 1e12, "unit": "TFLOP/s",
                     "speedup_vs_fp64": ms / mms, "refine_steps": rep["iterations"], "converged": rep["done"],
                     "info": inf, "ls_backward_error": mbe, "equal_fp64_error": bool(mbe <= 50 * EPS)}
    out = base_line(args, qr_flops(m, n) / (ms / 1e3) / 1e12, ms, "f64",
                    {"workload": "FP64 tiled-QR least squares, tall-skinny %dx%d, nb=%d (%dx%d tiles), "
                                 "N(0,1) entries, seed 1" % (m, n, nb, -(-m // nb), -(-n // nb)),
                     "m": m, "n": n, "nb": nb, "ib": args.ib, "tree": args.tree,
                     "kernels": args.kernels, "precision": "plain FP64"})
    out["executor_ms"] = kms
    out["ls_backward_error"] = be
    out["mixed_precision"] = mixed
    if not args.no_tree_compare:
        # the five trees of the thesis on identical inputs (FP64 lstsq, same nb)
        trees = {}
        for tr in ["flat", "binary", "fibonacci", "greedy", "grasap"]:
            ot = T.default_opts(nb=nb, ib=args.ib, tree=tr, kernels=args.kernels, stripes=args.stripes)
            wt = T.lstsq_workspace(m, n, 1, ot, dev)
            tms, tkms, _ = timed(lambda: T.lstsq(A, b, ot, X=X, work=wt, info=info), 2, 1, torch, T)
            cp = T.tqr_tree_cp(tr, -(-m // nb), -(-n // nb), 0, T.TT if args.kernels == "tt" else T.HYBRID)
            trees[tr] = {"ms_per_step": tms, "value": qr_flops(m, n) / (tms / 1e3) / 1e12,
                         "critical_path_units": cp, "ls_backward_error": backward_error(X[:, 0].cpu().numpy())}
            log("tree %s: %.2f ms (critical path %d units)" % (tr, tms, cp))
        out["trees"] = trees
        # beyond the stated configuration: the learned selector's choice of
        # (tree, nb) for this shape, and the best of a small grid
        from paper_1303_3182_amd import selector as S
        tuned = {}
        if S.load_selector() is not None:
            ot = T.default_opts(tree="auto", kernels=args.kernels)
            tid, snb, sib = S.select(m, n)
            wt = T.lstsq_workspace(m, n, 1, ot, dev)
            tms, _, _ = timed(lambda: T.lstsq(A, b, ot, X=X, work=wt, info=info), 3, 1, torch, T)
            name = [k for k, v in T.TREES.items() if v == tid][0]
            tuned["selector"] = {"tree": name, "nb": snb, "ib": sib, "ms_per_step": tms,
                                 "value": qr_flops(m, n) / (tms / 1e3) / 1e12}
            S.set_selector(None)
        best = None
        for gnb in (128, 256):
            for gtr in ("greedy", "fibonacci"):
                for gk in ("tt", "hybrid"):
                    og = T.default_opts(nb=gnb, tree=gtr, kernels=gk)
                    wg = T.lstsq_workspace(m, n, 1, og, dev)
                    gms, _, _ = timed(lambda: T.lstsq(A, b, og, X=X, work=wg, info=info), 3, 1, torch, T)
                    if best is None or gms < best["ms_per_step"]:
                        best = {"nb": gnb, "tree": gtr, "kernels": gk, "ms_per_step": gms,
                                "value": qr_flops(m, n) / (gms / 1e3) / 1e12,
                                "ls_backward_error": backward_error(X[:, 0].cpu().numpy())}
        tuned["best_of_grid"] = best
        log("tuned: %s" % json.dumps(tuned))
        out["tuned"] = tuned
    wkey = "tall %dx%d nb=%d ib=%d %s %s lstsq" % (m, n, nb, args.ib, args.tree, args.kernels)
    out["roofline"] = roofline(qr_flops(m, n), kms,
                               "exec_persistent (least-squares task graph: factor, Q^T b, R x = c)",
                               recorded_traffic("traffic_lstsq_16384x2048_nb256.json", wkey)
                               if args.stripes == 0 else None)
    if not args.no_cpu_baseline:
        c = args.cpu_sample_cols
        log("cpu baseline: oracle on a %d-column sample" % c)
        out["cpu_baseline"] = oracle_qr_rate(
            A0[:, :c].copy(order="F"), "unblocked FP64 Householder QR of the first %d columns of the %dx%d "
                                       "workload matrix (%d x %d)" % (c, m, n, m, c))
    return out


# ------------------------------------------------------- DAG upper bound
def gamma_ub(T, torch, np, m, n, nrhs, opts, run_once, tree_name, param=0, family=None):
    """The thesis's upper-bound model (section "Experimental results"):
    gamma_ub = gamma_task T / max(T/P, cp), T the total work and cp the
    critical path in units of nb^3/3 flop (table tab.kernels weights),
    P the concurrent task slots (executor workgroups) and gamma_task the
    per-workgroup kernel rate, here measured from one traced launch of the
    same least-squares graph (factorization tasks' flops over their summed
    durations).  A second form replaces the unit weights by every task's
    measured duration: t_ub = max(W / P, longest measured path)."""
    nb = opts.nb
    p, q = -(-m // nb), -(-n // nb)
    tasks = T.debug_graph(m, n, opts, nrhs=nrhs, kind=3)
    off, succ = T.debug_succ(m, n, opts, nrhs=nrhs, kind=3)
    nt = len(tasks)
    buf = torch.zeros(4 * nt, dtype=torch.int64, device="cuda")
    T.debug_trace(buf.data_ptr(), nt)
    try:
        run_once()
        torch.cuda.synchronize()
    finally:
        T.debug_trace(None, 0)
    tr = buf.cpu().numpy().reshape(nt, 4)
    ticks_per_ms = float(T.wallclock_khz())
    d = (tr[:, 1] - tr[:, 0]).astype(np.float64) / ticks_per_ms  # ms
    kinds = np.array([t[0] for t in tasks])
    P = T.executor_grid(opts)
    unit = nb ** 3 / 3.0
    weights = {0: 4, 1: 6, 2: 2, 3: 6, 4: 12, 5: 6}
    # factorization tasks: the six kernels on A's own tile columns (j < q);
    # the right-hand side's updates and the solve are excluded from the rate
    fact = np.array([t[0] < 6 and t[4] < q for t in tasks])
    units = 6 * p * q * q - 2 * q ** 3
    cp_units = T.tqr_tree_cp(tree_name, p, q, param, T.TT if family is None else family)
    # a kernel split into column stripes is several tasks sharing its units
    parts = {}
    for t in tasks:
        key = (t[0], t[1], t[2], t[3], t[4])
        parts[key] = parts.get(key, 0) + 1
    task_units = np.array([weights.get(t[0], 0) / parts[(t[0], t[1], t[2], t[3], t[4])] for t in tasks])
    rate = task_units[fact].sum() * unit / d[fact].sum()  # flop per ms per workgroup
    t_model = max(units / P, cp_units) * unit / rate
    # measured-duration form: longest path through the graph (Kahn order)
    indeg = np.zeros(nt, dtype=np.int64)
    for e in succ:
        indeg[e] += 1
    ready = [t for t in range(nt) if indeg[t] == 0]
    finish = np.zeros(nt)
    while ready:
        t = ready.pop()
        finish[t] += d[t]
        for e in range(off[t], off[t + 1]):
            s_ = succ[e]
            finish[s_] = max(finish[s_], finish[t])
            indeg[s_] -= 1
            if indeg[s_] == 0:
                ready.append(s_)
    cp_meas = float(finish.max())
    W = float(d.sum())
    t_meas = max(W / P, cp_meas)
    flops = qr_flops(m, n)
    span = (tr[:, 1].max() - tr[:, 0].min()) / ticks_per_ms
    by_kind = {}
    names = ["GEQRT", "TSQRT", "TTQRT", "UNMQR", "TSMQR", "TTMQR", "TRSM", "GEMM", "TRSMT", "GEMMT"]
    for k in sorted(set(kinds.tolist())):
        sel = kinds == k
        by_kind[names[k]] = {"tasks": int(sel.sum()), "mean_us": float(d[sel].mean() * 1e3),
                             "total_ms": float(d[sel].sum())}
    # the ALAP derived bound (chapter "Scheduling of Cholesky
    # Factorization", equation eqn:alapbound) and the critical-path list
    # schedule of the executor's own factorization graph on P slots, in
    # units and converted to time with the same per-slot rate
    sb = T.tqr_schedule_bounds(m, n, opts, P)
    sched = {k: sb[k] for k in ("cp", "t_seq", "lost_area", "alap_bound", "list_makespan")}
    sched["alap_bound_ms"] = sb["alap_bound"] * unit / rate
    sched["list_schedule_ms"] = sb["list_makespan"] * unit / rate
    return {"P": P, "T_units": units, "cp_units": cp_units, "schedule_bounds_units": sched,
            "gamma_task_tflops_per_slot": rate / 1e9,
            "thesis_model": {"t_ub_ms": t_model, "gamma_ub": flops / (t_model / 1e3) / 1e12,
                             "bound": "T/P" if units / P >= cp_units else "cp"},
            "measured_dag": {"t_ub_ms": t_meas, "gamma_ub": flops / (t_meas / 1e3) / 1e12,
                             "work_over_P_ms": W / P, "critical_path_ms": cp_meas,
                             "bound": "T/P" if W / P >= cp_meas else "cp"},
            "traced_span_ms": float(span), "busy_fraction": W / (P * span), "per_kind": by_kind}


def backward_error_square(np, A0, b0, x):
    """Rigal-Gaches ||b - A x|| / (||A||_F ||x|| + ||b||), long double."""
    Al = A0.astype(np.longdouble)
    r = b0.astype(np.longdouble) - Al @ x.astype(np.longdouble)
    nA = np.sqrt(np.sum(Al * Al))
    xl, bl = x.astype(np.longdouble), b0.astype(np.longdouble)
    return float(np.sqrt(np.dot(r, r)) / (nA * np.sqrt(np.dot(xl, xl)) + np.sqrt(np.dot(bl, bl))))


# -------------------------------------------------------------------- square
def run_square(args, np, torch, T, synth):
    n, nb = args.square_n, args.square_nb
    tree, param, kernels, ib = args.square_tree, args.square_param, args.square_kernels, args.square_ib
    fam = T.TT if kernels == "tt" else T.HYBRID
    dev = torch.device("cuda:0")
    X = torch.empty((1, n), dtype=torch.float64, device=dev).t()
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    per_kappa = {}
    fp64 = None
    gub = None
    for kappa in args.kappas:
        t0 = time.perf_counter()
        A0, x0, b0 = synth.conditioned(n, kappa, 7)
        log("kappa %g: inputs in %.1f s" % (kappa, time.perf_counter() - t0))
        A = T.colmajor(A0, dev)
        b = T.colmajor(b0[:, None], dev)
        res = {}
        for dt in ["f64"] + list(args.mixed):
            o = T.default_opts(nb=nb, ib=ib, tree=tree, param=param, kernels=kernels, update_dtype=dt,
                               max_refine=args.max_refine)
            w = T.lstsq_workspace(n, n, 1, o, dev)
            # the FP64 solve is kappa-independent: its full timing is taken once
            steps = args.steps if (dt != "f64" or fp64 is None) else max(2, args.steps // 4)
            ms, kms, nl = timed(lambda: T.lstsq(A, b, o, X=X, work=w, info=info), steps, args.warmup, torch, T)
            x = X[:, 0].cpu().numpy()
            be = backward_error_square(np, A0, b0, x)
            rep = T.refine_report(w)
            res[dt] = {"ms_per_step": ms, "value": qr_flops(n, n) / (ms / 1e3) / 1e12, "executor_ms": kms,
                       "executor_launches_per_step": nl, "refine_steps": rep["iterations"],
                       "gmres_steps": rep["gmres_steps"], "krylov_steps": rep["krylov_steps"],
                       "converged": rep["done"], "info": int(info.item()), "backward_error": be,
                       "equal_fp64_error": bool(be <= 50 * EPS and int(info.item()) == 0)}
            if dt == "f64" and fp64 is None:
                fp64 = {"ms": ms, "kms": kms, "be": be, "info": int(info.item())}
                if args.cold_steps > 0:
                    fp64["cold"] = cold_cache_timing(np, torch, T, lambda: T.lstsq(A, b, o, X=X, work=w, info=info),
                                                     args.cold_steps)
                    log("cold caches: executor %.2f ms (warm %.2f ms)" % (fp64["cold"]["executor_ms"], kms))
                if not args.no_gamma_ub:
                    gub = gamma_ub(T, torch, np, n, n, 1, o, lambda: T.lstsq(A, b, o, X=X, work=w, info=info),
                                   tree, param, fam)
            log("kappa %g %s: %.2f ms, be %.2e, refine %d (gmres %d, krylov %d), info %d" %
                (kappa, dt, ms, be, rep["iterations"], rep["gmres_steps"], rep["krylov_steps"], int(info.item())))
        for dt in args.mixed:
            res[dt]["speedup_vs_fp64"] = res["f64"]["ms_per_step"] / res[dt]["ms_per_step"]
        per_kappa["%g" % kappa] = res
        del A, b
    if fp64["info"] != 0:
        raise SystemExit("executor reported info=%d" % fp64["info"])
    out = base_line(args, qr_flops(n, n) / (fp64["ms"] / 1e3) / 1e12, fp64["ms"], "f64",
                    {"workload": "FP64 tiled-QR least squares of square %dx%d systems with prescribed condition "
                                 "number (Haar U, V; log-spaced sigma; b = A x + 1e-6 N(0,1)), nb=%d (%dx%d tiles), "
                                 "%s, %s kernels" % (n, n, nb, -(-n // nb), -(-n // nb),
                                                     "PlasmaTree(BS=%d)" % param if tree == "plasma"
                                                     else tree + " tree",
                                                     "TS" if kernels == "hybrid" and tree == "flat"
                                                     else ("TS domains, TT merges" if kernels == "hybrid"
                                                           else kernels.upper())),
                     "n": n, "nb": nb, "ib": ib, "tree": tree, "param": param, "kernels": kernels,
                     "kappas": args.kappas, "precision": "plain FP64"})
    out["executor_ms"] = fp64["kms"]
    if "cold" in fp64:
        out["cold_cache"] = fp64["cold"]
    out["ls_backward_error"] = fp64["be"]
    out["per_kappa"] = per_kappa
    out["mixed_summary"] = {
        dt: {k: {"speedup_vs_fp64": per_kappa[k][dt]["speedup_vs_fp64"],
                 "equal_fp64_error": per_kappa[k][dt]["equal_fp64_error"]} for k in per_kappa}
        for dt in args.mixed}
    out["not_at_fp64_error"] = ["%s kappa=%s" % (dt, k) for k in per_kappa for dt in per_kappa[k]
                                if not per_kappa[k][dt]["equal_fp64_error"]]
    out["roofline"] = roofline(qr_flops(n, n), fp64["kms"],
                               "exec_persistent (least-squares task graph: factor, Q^T b, R x = c)",
                               recorded_traffic("traffic_lstsq_8192x8192.json",
                                                "square %d nb=%d ib=%d %s/%d %s lstsq" % (n, nb, ib, tree, param,
                                                                                          kernels)))
    if gub is not None:
        out["gamma_ub"] = gub
        out["roofline"]["gamma_ub"] = gub["measured_dag"]["gamma_ub"]
        out["roofline"]["frac_of_gamma_ub"] = out["roofline"]["achieved"] / gub["measured_dag"]["gamma_ub"]
    if not args.no_c2:
        out["c2_trees"] = c2_trees(args, np, torch, T, synth)
    if args.cholinv_n > 0:
        out["cholinv"] = cholinv_leg(args, np, torch, T)
    if args.zqr_m > 0:
        out["zqr"] = zqr_leg(args, np, torch, T)
    if not args.no_cpu_baseline:
        A0, _, _ = synth.conditioned(n, args.kappas[0], 7)
        c = args.cpu_sample_cols
        log("cpu baseline: oracle on an %dx%d column sample" % (n, c))
        out["cpu_baseline"] = oracle_qr_rate(A0[:, :c].copy(order="F"),
                                             "unblocked FP64 Householder QR of the first %d columns of the "
                                             "%dx%d kappa=%g matrix (%d x %d)" % (c, n, n, args.kappas[0], n, c))
    return out


def cholinv_leg(args, np, torch, T):
    """Tile Cholesky inversion (chapter "Cholesky Inversion") of an n x n
    SPD matrix, G G^T / n + I with G ~ N(0,1) (seeded), nb = 64, in place
    and with array renaming: time per inversion (executor launch, HIP
    events) and n^3 / t in TFLOP/s; accuracy as ||A X - I||_F / (||A||_F
    ||X||_F) in FP64."""
    n, nb = args.cholinv_n, 64
    rng = np.random.default_rng(9)
    G = rng.standard_normal((n, n))
    A0 = G @ G.T / n + np.eye(n)
    dev = torch.device("cuda:0")
    Ad = T.colmajor(A0, dev)
    A = Ad.clone()
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    out = {"workload": "tile Cholesky inversion of an %dx%d SPD matrix (G G^T/n + I, N(0,1), seed 9), nb=%d "
                       "(%dx%d tiles), steps pipelined, UDU loop order" % (n, n, nb, -(-n // nb), -(-n // nb)),
           "n": n, "nb": nb, "flops": float(n) ** 3}
    for name, variant in (("in_place", T.CHOLINV_INPLACE), ("renamed", T.CHOLINV_RENAMED)):
        nbytes = T.tqr_cholinv_work_size(n, nb, variant)
        work = torch.empty(nbytes, dtype=torch.uint8, device=dev)

        def step():
            A.copy_(Ad)
            T.cholinv(A, nb=nb, variant=variant, work=work, info=info)

        ms, kms, _ = timed(step, max(3, args.steps // 2), 1, torch, T)
        X = np.tril(A.cpu().numpy())
        X = X + np.tril(X, -1).T
        res = float(np.linalg.norm(A0 @ X - np.eye(n)) / (np.linalg.norm(A0) * np.linalg.norm(X)))
        tasks, cp_tasks, cp_w = T.tqr_cholinv_graph_stats(-(-n // nb), variant)
        out[name] = {"executor_ms": kms, "ms_per_step_with_copy": ms, "tflops": float(n) ** 3 / (kms / 1e3) / 1e12,
                     "info": int(info.item()), "residual": res, "tasks": tasks,
                     "critical_path_tasks": cp_tasks, "critical_path_units": cp_w}
        log("cholinv %s n=%d: %.3f ms (%.2f TFLOP/s), residual %.2e" %
            (name, n, kms, out[name]["tflops"], res))
    out["roofline"] = {"bound": "alu", "achieved": out["renamed"]["tflops"], "peak": PEAK_FP64_MFMA,
                       "unit": "TFLOP/s", "frac": out["renamed"]["tflops"] / PEAK_FP64_MFMA,
                       "note": "FP64 FMA vector rate equals the FP64 matrix rate on this chip"}
    return out


def zqr_leg(args, np, torch, T):
    """Double-complex tiled QR (the thesis's "z" workloads) of an m x n
    matrix with i.i.d. complex N(0,1) entries (seed 11), nb = 64, Greedy,
    TT kernels: time per factorization (executor launch, HIP events) and
    8 n^2 (m - n/3) / t in TFLOP/s (a complex multiply-add is 8 real flops,
    4 times the real count; the thesis states no convention for its complex
    runs)."""
    m, n, nb = args.zqr_m, args.zqr_n, 64
    rng = np.random.default_rng(11)
    A0 = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    dev = torch.device("cuda:0")
    Ad = T.zcolmajor(A0, dev)
    A = Ad.clone()
    o = T.default_opts(nb=nb, tree="greedy", kernels="tt")
    nbytes = T.tqr_zworkspace_size(m, n, 0, o)
    W = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)

    def step():
        A.copy_(Ad)
        T.zfactor(A, o, W=W, info=info)

    ms, kms, _ = timed(step, max(3, args.steps // 2), 1, torch, T)
    flops = 8.0 * n * n * (m - n / 3.0)
    # accuracy: the Gram residual ||R^H (R z) - A^H (A z)|| / ||A^H (A z)||
    R = np.triu(A.cpu().numpy()[:n, :n])
    z = np.random.default_rng(12).standard_normal(n)
    g = A0.conj().T @ (A0 @ z)
    gram = float(np.linalg.norm(R.conj().T @ (R @ z) - g) / np.linalg.norm(g))
    out = {"workload": "double-complex tiled QR of a %dx%d matrix, complex N(0,1) entries (seed 11), nb=%d "
                       "(%dx%d tiles), greedy tree, TT kernels" % (m, n, nb, -(-m // nb), -(-n // nb)),
           "m": m, "n": n, "nb": nb, "executor_ms": kms, "ms_per_step_with_copy": ms,
           "tflops": flops / (kms / 1e3) / 1e12, "flops": flops, "info": int(info.item()), "gram_residual": gram}
    out["roofline"] = {"bound": "alu", "achieved": out["tflops"], "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s",
                       "frac": out["tflops"] / PEAK_FP64_MFMA}
    log("zqr %dx%d: %.3f ms (%.2f TFLOP/s), gram residual %.2e" % (m, n, kms, out["tflops"], gram))
    return out


def c2_trees(args, np, torch, T, synth, m=16384, n=2048, nb=256):
    """FP64 least squares on 16384 x 2048 with the five trees on identical
    inputs (time per solve and the tree's tiled critical path)."""
    A0 = synth.gaussian(m, n, 1)
    b0 = synth.gaussian_rhs(m, 1, 1)
    dev = torch.device("cuda:0")
    A = T.colmajor(A0, dev)
    b = T.colmajor(b0, dev)
    X = torch.empty((1, n), dtype=torch.float64, device=dev).t()
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    out = {"workload": "FP64 least squares, 16384x2048, nb=256 (64x8 tiles), N(0,1), seed 1"}
    for tr in ["flat", "binary", "fibonacci", "greedy", "grasap"]:
        ot = T.default_opts(nb=nb, ib=32, tree=tr)
        wt = T.lstsq_workspace(m, n, 1, ot, dev)
        tms, tkms, _ = timed(lambda: T.lstsq(A, b, ot, X=X, work=wt, info=info), 3, 1, torch, T)
        cp = T.tqr_tree_cp(tr, -(-m // nb), -(-n // nb), 0, T.TT)
        out[tr] = {"ms_per_step": tms, "value": qr_flops(m, n) / (tms / 1e3) / 1e12, "critical_path_units": cp,
                   "info": int(info.item())}
        log("c2 tree %s: %.2f ms (critical path %d units)" % (tr, tms, cp))
    return out


# ------------------------------------------------------------------- batched
def run_batched(args, np, torch, T, synth):
    from oracle import householder as H
    dev = torch.device("cuda:0")
    shapes = synth.ragged_batch_shapes(args.batch, 0)
    As, Bs = synth.ragged_batch(shapes, 0, 1)
    flops = sum(qr_flops(m, n) for m, n in shapes)
    log("batch of %d problems, %.3g QR flops" % (len(shapes), flops))
    dA = [T.colmajor(a, dev) for a in As]
    dB = [T.colmajor(b, dev) for b in Bs]
    Xs = [torch.empty((1, n), dtype=torch.float64, device=dev).t() for _, n in shapes]
    info = torch.zeros(len(shapes), dtype=torch.int32, device=dev)
    results = {}
    for dt in ["f64"] + list(args.mixed):
        o = T.default_opts(tree="auto", update_dtype=dt, max_refine=20)
        tune_ms = T.autotune_batched(dA, dB, o, Xs=Xs)
        work = T.lstsq_batched_workspace(shapes, 1, o, dev)
        ms, kms, nl = timed(lambda: T.lstsq_batched(dA, dB, o, Xs=Xs, work=work, info=info), args.steps,
                            args.warmup, torch, T)
        bad = int((info != 0).sum().item())
        sample = list(range(0, len(shapes), max(1, len(shapes) // 16)))
        bes = [H.ls_backward_error(As[x], Bs[x][:, 0], Xs[x][:, 0].cpu().numpy()) for x in sample]
        reps = T.refine_reports(work, len(shapes)) if dt != "f64" else []
        results[dt] = {"ms_per_step": ms, "value": flops / (ms / 1e3) / 1e12, "executor_ms": kms,
                       "launches_per_step": nl, "nb": o.nb, "ib": o.ib,
                       "kernels": {T.TT: "tt", T.HYBRID: "ts"}.get(o.kernels, o.kernels),
                       "tree": [k for k, v in T.TREES.items() if v == o.tree][0] if o.tree in T.TREES.values()
                       else "per-problem", "tree_param": o.param, "autotune_best_ms": tune_ms,
                       "problems_with_info": bad, "max_backward_error_sample": max(bes),
                       "sample_problems": len(sample), "equal_fp64_error": bool(max(bes) <= 50 * EPS)}
        if reps:
            results[dt]["max_refine_steps"] = max(r["iterations"] for r in reps)
            results[dt]["converged"] = sum(r["done"] for r in reps)
        log("batched %s: nb=%d ib=%d kernels=%d tree=%d/%d %.2f ms/step (%.2f TFLOP/s), max be %.2e" %
            (dt, o.nb, o.ib, o.kernels, o.tree, o.param, ms, flops / (ms / 1e3) / 1e12, max(bes)))
    for dt in args.mixed:
        results[dt]["speedup_vs_fp64"] = results["f64"]["ms_per_step"] / results[dt]["ms_per_step"]
    lead = args.mixed[0] if args.mixed else "f64"
    r0 = results[lead]
    out = base_line(args, r0["value"], r0["ms_per_step"], lead,
                    {"workload": "batched ragged least squares: %d problems, m log-uniform [256, 8192], "
                                 "n log-uniform [32, 512], n <= m/2, N(0,1), seed 0; %s updates + FP64 "
                                 "refinement; autotuned nb/ib, kernel family and tree policy" % (len(shapes), lead),
                     "problems": len(shapes), "qr_flops": flops})
    out["per_dtype"] = results
    out["roofline"] = roofline(flops, r0["executor_ms"] * r0["launches_per_step"],
                               "exec_persistent (batched least-squares task graph; all executor launches "
                               "of one step)")
    if not args.no_cpu_baseline:
        x = int(np.argmax([m * n for m, n in shapes]))
        out["cpu_baseline"] = oracle_qr_rate(As[x].copy(order="F"),
                                             "unblocked FP64 Householder QR of the batch's largest problem "
                                             "(%d x %d)" % shapes[x])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["tall", "square", "batched"], default="square")
    ap.add_argument("--m", type=int, default=16384)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--square-n", type=int, default=8192)
    # square workload configuration (measured fastest among the trees, both
    # kernel families, PlasmaTree domain sizes and nb 64 / 128 / 256 on this
    # workload: PlasmaTree with TS domains of 48 tile rows and TT merges)
    ap.add_argument("--square-nb", type=int, default=128)
    ap.add_argument("--square-ib", type=int, default=32)
    ap.add_argument("--square-tree", default="plasma")
    ap.add_argument("--square-param", type=int, default=48)
    ap.add_argument("--square-kernels", default="hybrid")
    ap.add_argument("--kappas", type=float, nargs="*", default=[1e2, 1e5, 1e8])
    ap.add_argument("--cold-steps", type=int, default=3,
                    help="FP64 square solves timed after flushing the caches (0: none)")
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--ib", type=int, default=32)
    ap.add_argument("--tree", default="greedy")
    ap.add_argument("--no-tree-compare", action="store_true",
                    help="skip timing the five trees on the tall-skinny workload")
    ap.add_argument("--kernels", default="tt")
    ap.add_argument("--stripes", type=int, default=0)
    ap.add_argument("--cpu-sample-cols", type=int, default=256)
    ap.add_argument("--no-c2", action="store_true", help="skip the 16384x2048 five-tree comparison")
    ap.add_argument("--no-gamma-ub", action="store_true", help="skip the traced launch of the DAG bound")
    ap.add_argument("--cholinv-n", type=int, default=4096,
                    help="size of the tile Cholesky inversion leg of the default run (0: skip)")
    ap.add_argument("--zqr-m", type=int, default=8192, help="rows of the double-complex QR leg (0: skip)")
    ap.add_argument("--zqr-n", type=int, default=2048, help="columns of the double-complex QR leg")
    ap.add_argument("--max-refine", type=int, default=20)
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

    torch.cuda.set_device(0)
    run = {"tall": run_tall, "square": run_square, "batched": run_batched}[args.workload]
    print(json.dumps(run(args, np, torch, T, synth)))


if __name__ == "__main__":
    main()
