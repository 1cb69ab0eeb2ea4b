"""The learned tree / tile-size selector: bindings of the network kernels
(forward, gradient, Adam, full-batch fitting; all on the GPU), feature
vectors, registration of a trained network for TQR_AUTO, and the timing
collection and training procedure that produces the shipped weights
(selector_weights.npy).

Run as a module on a GPU machine to (re)train:
    python -m paper_1303_3182_amd.selector --train 2000 --heldout 200
"""
import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import _binding as B
from .api import _stream

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_weights.npy")
TREES = ["flat", "binary", "fibonacci", "greedy", "grasap"]
NBS = [64, 128, 256]
IB_OF = {64: 32, 128: 32, 256: 32}


def n_params():
    return int(B.lib().tqr_mlp_params())


def n_features():
    return int(B.lib().tqr_mlp_features())


def features(m, n, nb, tree, batch=1):
    out = (ctypes.c_float * n_features())()
    t = B.TREES[tree] if isinstance(tree, str) else tree
    B._check(B.lib().tqr_mlp_features_of(m, n, nb, t, batch, out), "tqr_mlp_features_of")
    return np.array(out[:], dtype=np.float32)


def init_params(seed=0, device="cuda"):
    """Random initial weights (seeded): N(0, 1/fan_in) weights, zero biases."""
    rng = np.random.default_rng(seed)
    H, F = 64, n_features()
    w = np.concatenate([rng.standard_normal(H * F) / math.sqrt(F), np.zeros(H),
                        rng.standard_normal(H * H) / math.sqrt(H), np.zeros(H),
                        rng.standard_normal(H) / math.sqrt(H), np.zeros(1)]).astype(np.float32)
    assert w.size == n_params()
    return torch.from_numpy(w).to(device)


def forward(params, X):
    X = X.contiguous()
    y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    B._check(B.lib().tqr_mlp_forward(params.data_ptr(), X.data_ptr(), X.shape[0], y.data_ptr(), _stream()),
             "tqr_mlp_forward")
    return y


def _work(batch, device):
    return torch.empty(int(B.lib().tqr_mlp_work_size(batch)), dtype=torch.uint8, device=device)


def grad(params, X, t):
    """(gradient of mean((y - t)^2), loss) computed by the GPU kernels."""
    X = X.contiguous()
    g = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    w = _work(X.shape[0], X.device)
    B._check(B.lib().tqr_mlp_grad(params.data_ptr(), X.data_ptr(), t.data_ptr(), X.shape[0], g.data_ptr(),
                                  loss.data_ptr(), w.data_ptr(), w.numel(), _stream()), "tqr_mlp_grad")
    return g, loss


def adam(params, g, m1, m2, step, lr):
    B._check(B.lib().tqr_mlp_adam(params.data_ptr(), g.data_ptr(), m1.data_ptr(), m2.data_ptr(), step, lr,
                                  _stream()), "tqr_mlp_adam")


def fit(params, X, t, epochs, lr):
    """Full-batch Adam on the GPU; returns the loss before each step."""
    X = X.contiguous()
    hist = torch.empty(max(epochs, 1), dtype=torch.float32, device=X.device)
    w = _work(X.shape[0], X.device)
    B._check(B.lib().tqr_mlp_fit(params.data_ptr(), X.data_ptr(), t.data_ptr(), X.shape[0], epochs, lr,
                                 hist.data_ptr(), w.data_ptr(), w.numel(), _stream()), "tqr_mlp_fit")
    return hist[:epochs]


def set_selector(params):
    """Registers a trained network for TQR_AUTO (None clears it)."""
    torch.cuda.synchronize()
    B._check(B.lib().tqr_set_selector(None if params is None else params.data_ptr()), "tqr_set_selector")


def load_selector(path=WEIGHTS, device="cuda"):
    """Loads the shipped weights (if present) and registers them; returns the
    parameter tensor or None."""
    if not os.path.exists(path):
        return None
    w = np.load(path, allow_pickle=False).astype(np.float32)
    p = torch.from_numpy(w).to(device)
    set_selector(p)
    return p


def select(m, n, batch=1):
    """(tree id, nb, ib) that TQR_AUTO would use for an m x n problem."""
    t, nb, ib = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    B._check(B.lib().tqr_select(m, n, batch, ctypes.byref(t), ctypes.byref(nb), ctypes.byref(ib)), "tqr_select")
    return t.value, nb.value, ib.value


# ------------------------------------------------------- timing collection
def time_factor(m, n, nb, tree, reps=2, seed=0, device="cuda"):
    """Milliseconds of one FP64 tqr_factor_ex of an m x n N(0,1) matrix with
    the given tile size and tree (median of reps launches, after a warm-up
    that builds the plan)."""
    from . import api
    g = torch.Generator(device=device).manual_seed(seed)
    A0 = torch.randn((n, m), dtype=torch.float64, device=device, generator=g).t()
    A = A0.clone()
    opts = B.default_opts(nb=nb, ib=IB_OF[nb], tree=tree)
    W = api.workspace(m, n, 0, opts, device)
    api.factor(A, opts, T=W)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        A.copy_(A0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        api.factor(A, opts, T=W)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def random_shapes(count, seed, m_range=(1024, 262144), n_max=8192, max_elems=1 << 25):
    """m log-uniform in m_range, n log-uniform in [64, min(n_max, m)],
    keeping m * n <= max_elems (a bound on the timing budget)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        m = int(round(math.exp(rng.uniform(math.log(m_range[0]), math.log(m_range[1])))))
        n = int(round(math.exp(rng.uniform(math.log(64), math.log(min(n_max, m))))))
        if m * n <= max_elems:
            out.append((m, n))
    return out


def collect(shapes, seed, log=print):
    """One timed (shape, tree, nb) sample per shape, tree and nb drawn at
    random: features X and log(ms) targets."""
    rng = np.random.default_rng(seed)
    X, y, meta = [], [], []
    t0 = time.time()
    for i, (m, n) in enumerate(shapes):
        tree = TREES[rng.integers(len(TREES))]
        nb = NBS[rng.integers(len(NBS))]
        ms = time_factor(m, n, nb, tree, seed=i)
        X.append(features(m, n, nb, tree))
        y.append(math.log(ms))
        meta.append((m, n, nb, tree, ms))
        if i % 100 == 0:
            log("sample %d/%d (%.0f s): %dx%d nb=%d %s %.2f ms" % (i, len(shapes), time.time() - t0, m, n, nb,
                                                                    tree, ms))
    return np.array(X, dtype=np.float32), np.array(y, dtype=np.float32), meta


def evaluate(params, shapes, log=print):
    """For each held-out shape: time every (tree, nb) candidate, the
    fallback GrASAP at nb = 256 and the network's pick; returns a dict of
    totals and per-shape rows."""
    set_selector(params)
    rows = []
    for i, (m, n) in enumerate(shapes):
        grid = {(t, nb): time_factor(m, n, nb, t, seed=10_000 + i) for t in TREES for nb in NBS}
        tid, nb, ib = select(m, n)
        pick = (TREES[[B.TREES[t] for t in TREES].index(tid)], nb)
        best = min(grid, key=grid.get)
        rows.append({"m": m, "n": n, "pick": pick, "pick_ms": grid[pick], "fallback_ms": grid[("grasap", 256)],
                     "best": best, "best_ms": grid[best]})
        if i % 20 == 0:
            log("held-out %d/%d: %dx%d pick %s %.2f ms, fallback %.2f, best %s %.2f" % (
                i, len(shapes), m, n, pick, grid[pick], grid[("grasap", 256)], best, grid[best]))
        # baseline without timing: Greedy at the tile size whose critical
        # path (units of nb^3/3, table tab.kernels weights) is shortest in time
        cp_nb = min(NBS, key=lambda b: B.tqr_tree_cp("greedy", -(-m // b), -(-n // b)) * float(b) ** 3)
        rows[-1]["greedy_cp_nb"] = cp_nb
        rows[-1]["greedy_cp_ms"] = grid[("greedy", cp_nb)]
        rows[-1]["grid"] = {"%s/%d" % k: v for k, v in grid.items()}
    tot = {k: float(sum(r[k] for r in rows)) for k in ("pick_ms", "fallback_ms", "best_ms", "greedy_cp_ms")}
    # the single (tree, nb) with the smallest total over these shapes: the
    # best any constant choice could do (chosen with hindsight)
    const_tot = {key: sum(r["grid"][key] for r in rows) for key in rows[0]["grid"]} if rows else {}
    best_const = min(const_tot, key=const_tot.get) if rows else None
    gains = [r["fallback_ms"] / r["pick_ms"] for r in rows]
    regret = [r["pick_ms"] / r["best_ms"] for r in rows]
    return {"shapes": len(rows), "total_pick_ms": tot["pick_ms"], "total_fallback_ms": tot["fallback_ms"],
            "total_best_ms": tot["best_ms"], "speedup_total": tot["fallback_ms"] / tot["pick_ms"],
            "total_greedy_cp_nb_ms": tot["greedy_cp_ms"], "best_constant": best_const,
            "total_best_constant_ms": float(const_tot[best_const]) if rows else None,
            "geomean_speedup": float(np.exp(np.mean(np.log(gains)))),
            "geomean_regret": float(np.exp(np.mean(np.log(regret)))), "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--heldout", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--max-elems", type=int, default=1 << 25)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default=None)
    ap.add_argument("--eval-only", action="store_true", help="evaluate the weights in --out, no training")
    args = ap.parse_args()

    def log(msg):
        sys.stderr.write("[selector] %s\n" % msg)
        sys.stderr.flush()

    dev = "cuda"
    if args.eval_only:
        params = torch.from_numpy(np.load(args.out, allow_pickle=False)).to(dev)
        shapes, meta, hist = [], [], np.array([float("nan")])
    else:
        shapes = random_shapes(args.train, 1, max_elems=args.max_elems)
        X, y, meta = collect(shapes, 2, log)
        params = init_params(0, dev)
        Xd = torch.from_numpy(X).to(dev)
        yd = torch.from_numpy(y).to(dev)
        hist = fit(params, Xd, yd, args.epochs, args.lr).cpu().numpy()
        log("training loss: first %.4f, last %.4f" % (hist[0], hist[-1]))
        np.save(args.out, params.cpu().numpy(), allow_pickle=False)
    held = random_shapes(args.heldout, 3, max_elems=args.max_elems)
    ev = evaluate(params, held, log)
    log("held-out: pick %.1f ms, fallback %.1f ms, best %.1f ms, best constant %s %.1f ms, greedy at cp-best nb "
        "%.1f ms; speedup %.3f, geomean %.3f, regret %.3f" % (
            ev["total_pick_ms"], ev["total_fallback_ms"], ev["total_best_ms"], ev["best_constant"],
            ev["total_best_constant_ms"], ev["total_greedy_cp_nb_ms"], ev["speedup_total"],
            ev["geomean_speedup"], ev["geomean_regret"]))
    rep = {"train_samples": len(shapes), "epochs": args.epochs, "lr": args.lr, "loss_first": float(hist[0]),
           "loss_last": float(hist[-1]), "heldout": {k: v for k, v in ev.items() if k != "rows"}}
    if args.report:
        with open(args.report, "w") as f:
            json.dump({"summary": rep, "rows": ev["rows"], "train": meta}, f)
    print(json.dumps(rep))


if __name__ == "__main__":
    main()
