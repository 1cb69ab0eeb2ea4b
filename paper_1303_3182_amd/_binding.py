"""ctypes view of libtqr.so: one Python function per C entry point, same
names and argument order as include/tqr.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libtqr.so")

FLAT, BINARY, FIBONACCI, GREEDY, GRASAP, PLASMA, ASAP, AUTO = 0, 1, 2, 3, 4, 5, 6, 100
TREES = {"flat": FLAT, "binary": BINARY, "fibonacci": FIBONACCI, "greedy": GREEDY,
         "grasap": GRASAP, "plasma": PLASMA, "asap": ASAP, "auto": AUTO}
TT, HYBRID = 0, 1
F64, F32, BF16 = 0, 1, 2
EXEC_PERSISTENT, EXEC_SEQUENTIAL = 0, 1
REFINE_AUTO, REFINE_CLASSICAL, REFINE_GMRES = 0, 1, 2
PRIO_LIST, PRIO_BOTTOM, PRIO_STATIC = 0, 1, 2


class TqrError(RuntimeError):
    pass


class Opts(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int32), ("ib", ctypes.c_int32), ("tree", ctypes.c_int32),
                ("kernels", ctypes.c_int32), ("param", ctypes.c_int32),
                ("update_dtype", ctypes.c_int32), ("exec", ctypes.c_int32),
                ("stripes", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("priority", ctypes.c_int32), ("refine_method", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("refine_tol", ctypes.c_double)]


_lib = None


def library_path():
    return _LIB_PATH


def lib():
    """The loaded libtqr.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise TqrError("libtqr.so is not built (run __graft_entry__.build() or "
                           "python -m paper_1303_3182_amd.build)")
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        op = ctypes.POINTER(Opts)
        i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
        vpp = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "tqr_default_opts": (None, [op]),
            "tqr_workspace_size": (sz, [i64, i64, i64, op]),
            "tqr_factor": (ctypes.c_int, [i64, i64, i32, i32, vp, vp, vp]),
            "tqr_factor_ex": (ctypes.c_int, [i64, i64, vp, i64, vp, sz, op, vp, vp]),
            "tqr_apply_qt": (ctypes.c_int, [i64, i64, vp, i64, vp, sz, i64, vp, i64, op, vp, vp]),
            "tqr_solve_r": (ctypes.c_int, [i64, i64, vp, i64, vp, sz, i64, vp, i64, op, vp, vp]),
            "tqr_lstsq_work_size": (sz, [i64, i64, i64, op]),
            "tqr_lstsq": (ctypes.c_int, [i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, sz, op, vp, vp]),
            "tqr_lstsq_noalloc": (ctypes.c_int, [i64, i64, i64, vp, i64, vp, i64, vp, i64, op, vp, vp]),
            "tqr_tree_list": (i64, [i32, i32, i32, i32, i32p, i32p, i32p, i64]),
            "tqr_tree_cp": (i64, [i32, i32, i32, i32, i32, i64p, i64p]),
            "tqr_graph_stats": (ctypes.c_int, [i64, i64, op, i64p, i64p]),
            "tqr_schedule_bounds": (ctypes.c_int, [i64, i64, op, i32, ctypes.POINTER(ctypes.c_double)]),
            "tqr_cholinv_work_size": (sz, [i64, i32, i32]),
            "tqr_zworkspace_size": (sz, [i64, i64, i64, op]),
            "tqr_zfactor": (ctypes.c_int, [i64, i64, vp, i64, vp, sz, op, vp, vp]),
            "tqr_zapply_qh": (ctypes.c_int, [i64, i64, vp, i64, vp, sz, i64, vp, i64, op, vp, vp]),
            "tqr_cholinv": (ctypes.c_int, [i64, vp, i64, i32, i32, vp, sz, vp, vp]),
            "tqr_cholinv_graph_stats": (ctypes.c_int, [i32, i32, i64p, ctypes.POINTER(ctypes.c_double),
                                                       ctypes.POINTER(ctypes.c_double)]),
            "tqr_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "tqr_lstsq_batched_work_size": (sz, [i32, i64p, i64p, i64, op]),
            "tqr_lstsq_batched": (ctypes.c_int, [i32, i64p, i64p, i64, vpp, i64p, vpp, i64p, vpp, i64p, vp, sz, op,
                                                 vp, vp]),
            "tqr_autotune_batched": (ctypes.c_int, [i32, i64p, i64p, i64, vpp, i64p, vpp, i64p, vpp, i64p, vp, sz,
                                                    op, ctypes.POINTER(ctypes.c_float), vp]),
            "tqr_mlp_params": (i32, []),
            "tqr_mlp_features": (i32, []),
            "tqr_mlp_features_of": (ctypes.c_int, [i64, i64, i32, i32, i32, ctypes.POINTER(ctypes.c_float)]),
            "tqr_mlp_work_size": (sz, [i64]),
            "tqr_mlp_forward": (ctypes.c_int, [vp, vp, i64, vp, vp]),
            "tqr_mlp_grad": (ctypes.c_int, [vp, vp, vp, i64, vp, vp, vp, sz, vp]),
            "tqr_mlp_adam": (ctypes.c_int, [vp, vp, vp, vp, i64, ctypes.c_float, vp]),
            "tqr_mlp_fit": (ctypes.c_int, [vp, vp, vp, i64, i32, ctypes.c_float, vp, vp, sz, vp]),
            "tqr_set_selector": (ctypes.c_int, [vp]),
            "tqr_select": (ctypes.c_int, [i64, i64, i32, i32p, i32p, i32p]),
            "tqr_debug_trace": (None, [vp, i64]),
            "tqr_debug_spin_limit": (None, [i64]),
            "tqr_executor_grid": (ctypes.c_int, [op]),
            "tqr_wallclock_khz": (i64, []),
            "tqr_debug_timing": (None, [i32]),
            "tqr_debug_timing_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), i64p]),
            "tqr_debug_graph": (ctypes.c_int, [i64, i64, i64, i32, op, i32p, i64]),
            "tqr_debug_succ": (ctypes.c_int, [i64, i64, i64, i32, op, i32p, i32p, i64]),
            "tqr_debug_ready": (ctypes.c_int, [i64, i64, i64, i32, op, i32p, i64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


REFINE_HISTORY = 24  # TQR_REFINE_HISTORY


def _check(rc, what):
    if rc != 0:
        msg = lib().tqr_strerror(rc).decode()
        raise TqrError("%s failed: %d (%s)" % (what, rc, msg))
    return rc


def _opts_ptr(o):
    return None if o is None else ctypes.byref(o)


def default_opts(**kw):
    o = Opts()
    lib().tqr_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "tree" and isinstance(v, str):
            v = TREES[v]
        if k == "kernels" and isinstance(v, str):
            v = {"tt": TT, "hybrid": HYBRID, "ts": HYBRID}[v]
        if k == "update_dtype" and isinstance(v, str):
            v = {"f64": F64, "f32": F32, "bf16": BF16}[v]
        if k == "refine_method" and isinstance(v, str):
            v = {"auto": REFINE_AUTO, "classical": REFINE_CLASSICAL, "gmres": REFINE_GMRES}[v]
        if k == "priority" and isinstance(v, str):
            v = {"list": PRIO_LIST, "bottom": PRIO_BOTTOM, "static": PRIO_STATIC}[v]
        setattr(o, k, v)
    return o


def tqr_workspace_size(m, n, nrhs=0, opts=None):
    return int(lib().tqr_workspace_size(m, n, nrhs, _opts_ptr(opts)))


def tqr_factor(m, n, nb, tree, A, T, stream):
    return _check(lib().tqr_factor(m, n, nb, tree, A, T, stream), "tqr_factor")


def tqr_factor_ex(m, n, A, lda, T, t_bytes, opts, info, stream):
    return _check(lib().tqr_factor_ex(m, n, A, lda, T, t_bytes, _opts_ptr(opts), info, stream),
                  "tqr_factor_ex")


def tqr_apply_qt(m, n, A, lda, T, t_bytes, nrhs, B, ldb, opts, info, stream):
    return _check(lib().tqr_apply_qt(m, n, A, lda, T, t_bytes, nrhs, B, ldb, _opts_ptr(opts), info,
                                     stream), "tqr_apply_qt")


def tqr_solve_r(m, n, A, lda, T, t_bytes, nrhs, B, ldb, opts, info, stream):
    return _check(lib().tqr_solve_r(m, n, A, lda, T, t_bytes, nrhs, B, ldb, _opts_ptr(opts), info,
                                    stream), "tqr_solve_r")


def tqr_lstsq_work_size(m, n, nrhs, opts=None):
    return int(lib().tqr_lstsq_work_size(m, n, nrhs, _opts_ptr(opts)))


def tqr_lstsq(m, n, nrhs, A, lda, B, ldb, X, ldx, work, work_bytes, opts, info, stream):
    return _check(lib().tqr_lstsq(m, n, nrhs, A, lda, B, ldb, X, ldx, work, work_bytes,
                                  _opts_ptr(opts), info, stream), "tqr_lstsq")


def tqr_lstsq_noalloc(m, n, nrhs, A, lda, B, ldb, X, ldx, opts, info, stream):
    return _check(lib().tqr_lstsq_noalloc(m, n, nrhs, A, lda, B, ldb, X, ldx, _opts_ptr(opts), info, stream),
                  "tqr_lstsq_noalloc")


def tqr_tree_list(tree, p, q, param=0):
    """1-based (i, piv, k) triples of the elimination list (host only)."""
    if isinstance(tree, str):
        tree = TREES[tree]
    L = lib()
    n = L.tqr_tree_list(tree, p, q, param, None, None, None, 0)
    if n < 0:
        raise TqrError("tqr_tree_list: bad arguments (%d)" % n)
    a = (ctypes.c_int32 * max(n, 1))()
    b = (ctypes.c_int32 * max(n, 1))()
    c = (ctypes.c_int32 * max(n, 1))()
    L.tqr_tree_list(tree, p, q, param, a, b, c, n)
    return [(a[e], b[e], c[e]) for e in range(n)]


def tqr_tree_cp(tree, p, q, param=0, kernels=TT, want_zero=False):
    """Critical path (units nb^3/3); optionally (cp, zero_times p x q, counts)."""
    if isinstance(tree, str):
        tree = TREES[tree]
    zt = (ctypes.c_int64 * (p * q))()
    cnt = (ctypes.c_int64 * 6)()
    cp = lib().tqr_tree_cp(tree, p, q, param, kernels, zt, cnt)
    if cp < 0:
        raise TqrError("tqr_tree_cp: bad arguments (%d)" % cp)
    if not want_zero:
        return int(cp)
    rows = [[zt[i * q + k] for k in range(q)] for i in range(p)]
    return int(cp), rows, list(cnt)


def tqr_graph_stats(m, n, opts=None):
    nt, ne = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().tqr_graph_stats(m, n, _opts_ptr(opts), ctypes.byref(nt), ctypes.byref(ne)),
           "tqr_graph_stats")
    return nt.value, ne.value


def tqr_schedule_bounds(m, n, opts=None, P=1):
    """Bounded-processor analysis of the factorization graph on P
    processors: dict of cp, t_seq, lost_area, alap_bound and list_makespan
    (units nb^3/3)."""
    out = (ctypes.c_double * 5)()
    _check(lib().tqr_schedule_bounds(m, n, _opts_ptr(opts), P, out), "tqr_schedule_bounds")
    return dict(zip(("cp", "t_seq", "lost_area", "alap_bound", "list_makespan"), list(out)))


CHOLINV_INPLACE, CHOLINV_RENAMED, CHOLINV_UUU = 0, 1, 2


def tqr_zworkspace_size(m, n, nrhs=0, opts=None):
    return int(lib().tqr_zworkspace_size(m, n, nrhs, _opts_ptr(opts)))


def tqr_zfactor(m, n, A, lda, W, w_bytes, opts, info, stream):
    return _check(lib().tqr_zfactor(m, n, A, lda, W, w_bytes, _opts_ptr(opts), info, stream), "tqr_zfactor")


def tqr_zapply_qh(m, n, A, lda, W, w_bytes, nrhs, B, ldb, opts, info, stream):
    return _check(lib().tqr_zapply_qh(m, n, A, lda, W, w_bytes, nrhs, B, ldb, _opts_ptr(opts), info, stream),
                  "tqr_zapply_qh")


def tqr_cholinv_work_size(n, nb=64, variant=CHOLINV_INPLACE):
    return int(lib().tqr_cholinv_work_size(n, nb, variant))


def tqr_cholinv(n, A, lda, nb, variant, work, work_bytes, info, stream):
    return _check(lib().tqr_cholinv(n, A, lda, nb, variant, work, work_bytes, info, stream), "tqr_cholinv")


def tqr_cholinv_graph_stats(t, variant=CHOLINV_INPLACE):
    """(tasks, critical path in tasks, weighted critical path in nb^3/3) of
    the inversion's graph for t x t tiles (host only)."""
    nt = ctypes.c_int64()
    cpt, cpw = ctypes.c_double(), ctypes.c_double()
    _check(lib().tqr_cholinv_graph_stats(t, variant, ctypes.byref(nt), ctypes.byref(cpt), ctypes.byref(cpw)),
           "tqr_cholinv_graph_stats")
    return nt.value, cpt.value, cpw.value


def debug_timing(enable):
    """Start (True) or stop (False) HIP-event timing of every executor launch."""
    lib().tqr_debug_timing(1 if enable else 0)


def debug_timing_read():
    """(total milliseconds, number of launches) of the executor launches
    timed since debug_timing(True); waits for them to finish."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(lib().tqr_debug_timing_read(ctypes.byref(ms), ctypes.byref(cnt)), "tqr_debug_timing_read")
    return ms.value, cnt.value


def debug_trace(buf_ptr, cap):
    """Record per-task clock stamps into a device int64 buffer (debug)."""
    lib().tqr_debug_trace(buf_ptr, cap)


def executor_grid(opts=None):
    """Workgroups of the persistent executor launch (concurrent task slots)."""
    g = lib().tqr_executor_grid(_opts_ptr(opts))
    if g < 0:
        _check(g, "tqr_executor_grid")
    return g


def wallclock_khz():
    """Rate of the device wall clock of the trace stamps, in kHz."""
    k = lib().tqr_wallclock_khz()
    if k <= 0:
        _check(int(k), "tqr_wallclock_khz")
    return int(k)


def debug_spin_limit(ticks):
    """Watchdog limit of later executor launches in wall-clock ticks (0 =
    the default of 30 s); debug and failure-handling tests only."""
    lib().tqr_debug_spin_limit(int(ticks))


def debug_graph(m, n, opts=None, nrhs=0, kind=0):
    """Task table of a plan as a list of (kind, i, piv, k, j, stripe, nsucc, npred)."""
    L = lib()
    nt = L.tqr_debug_graph(m, n, nrhs, kind, _opts_ptr(opts), None, 0)
    if nt < 0:
        raise TqrError("tqr_debug_graph failed (%d)" % nt)
    buf = (ctypes.c_int32 * (8 * max(nt, 1)))()
    L.tqr_debug_graph(m, n, nrhs, kind, _opts_ptr(opts), buf, nt)
    return [tuple(buf[8 * t:8 * t + 8]) for t in range(nt)]


def debug_ready(m, n, opts=None, nrhs=0, kind=0):
    """Initially ready tasks of a plan in queue order (with the static order:
    every task, in the order the executor hands them out)."""
    L = lib()
    nt = len(debug_graph(m, n, opts, nrhs, kind))
    ready = (ctypes.c_int32 * max(nt, 1))()
    nr = L.tqr_debug_ready(m, n, nrhs, kind, _opts_ptr(opts), ready, nt)
    if nr < 0:
        raise TqrError("tqr_debug_ready failed (%d)" % nr)
    return list(ready[:nr])


def debug_succ(m, n, opts=None, nrhs=0, kind=0):
    """Successor lists (CSR offsets, successors) of a plan."""
    L = lib()
    tasks = debug_graph(m, n, opts, nrhs, kind)
    ne = sum(t[6] for t in tasks)
    off = (ctypes.c_int32 * (len(tasks) + 1))()
    succ = (ctypes.c_int32 * max(ne, 1))()
    L.tqr_debug_succ(m, n, nrhs, kind, _opts_ptr(opts), off, succ, ne)
    return list(off), list(succ)
