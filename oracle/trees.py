"""ORACLE -- test infrastructure only (see oracle/__init__).

Python view of the plain-C scheduling oracle ``tiledqr_lists.c``:
elimination lists (thesis section "Elimination lists"), the coarse-grain
model (section "Coarse-grain algorithms") and the tiled model with the
kernel weights of table tab.kernels (section "Tiled algorithms").
Row/column indices are 1-based, as in the thesis.
"""
import ctypes

import numpy as np

from .build import build_oracle

FLAT, BINARY, FIBONACCI, GREEDY, GRASAP, PLASMA, ASAP = range(7)
TT, HYBRID = 0, 1
KERNELS = ("GEQRT", "TSQRT", "TTQRT", "UNMQR", "TSMQR", "TTMQR")
NAMES = {"flat": FLAT, "binary": BINARY, "fibonacci": FIBONACCI, "greedy": GREEDY,
         "grasap": GRASAP, "plasma": PLASMA, "asap": ASAP}

_lib = None


def _L():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_oracle())
        i32p = ctypes.POINTER(ctypes.c_int)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.orc_list.argtypes = [ctypes.c_int] * 4 + [i32p, i32p, i32p, ctypes.c_int]
        lib.orc_list.restype = ctypes.c_int
        lib.orc_tiled.argtypes = [ctypes.c_int] * 4 + [i32p] * 3 + [i64p] * 4
        lib.orc_tiled.restype = ctypes.c_int64
        lib.orc_tree_cp.argtypes = [ctypes.c_int] * 5
        lib.orc_tree_cp.restype = ctypes.c_int64
        lib.orc_coarse.argtypes = [ctypes.c_int] * 3 + [i32p] * 4
        lib.orc_coarse.restype = ctypes.c_int
        lib.orc_fib_coarse.argtypes = [ctypes.c_int, ctypes.c_int, i32p]
        lib.orc_fib_coarse.restype = None
        _lib = lib
    return _lib


def _tree_id(tree):
    return NAMES[tree] if isinstance(tree, str) else int(tree)


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _p64(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def elimination_list(tree, p, q, param=0):
    """List of (i, piv, k) for a p x q tile matrix, in list order.

    ``param`` is the domain size BS for PlasmaTree and i for GrASAP(i)."""
    lib = _L()
    t = _tree_id(tree)
    n = lib.orc_list(t, p, q, param, None, None, None, 0)
    if n < 0:
        raise ValueError("bad tree/shape")
    a = np.zeros((3, max(n, 1)), dtype=np.int32)
    lib.orc_list(t, p, q, param, _p32(a[0]), _p32(a[1]), _p32(a[2]), n)
    return [tuple(int(v) for v in a[:, e]) for e in range(n)]


def tiled(p, q, elist, mode=TT):
    """Tiled execution of a list (unbounded processors).

    Returns a dict with the critical path ``cp`` and p x q arrays (index
    [i-1, k-1]) ``zero`` (end of the kernel that zeroes tile (i,k)),
    ``geqrt`` (end of GEQRT(i,k)), ``upd`` (end of the update of column k+1
    that follows the zeroing of (i,k)) and the kernel ``counts``."""
    lib = _L()
    a = np.array(elist, dtype=np.int32).reshape(-1, 3).T.copy() if elist else np.zeros((3, 1), np.int32)
    n = len(elist)
    zero = np.zeros(p * q, dtype=np.int64)
    geq = np.zeros(p * q, dtype=np.int64)
    upd = np.zeros(p * q, dtype=np.int64)
    cnt = np.zeros(6, dtype=np.int64)
    cp = lib.orc_tiled(p, q, mode, n, _p32(a[0]), _p32(a[1]), _p32(a[2]),
                       _p64(zero), _p64(geq), _p64(upd), _p64(cnt))
    return {"cp": int(cp), "zero": zero.reshape(p, q), "geqrt": geq.reshape(p, q),
            "upd": upd.reshape(p, q), "counts": dict(zip(KERNELS, (int(c) for c in cnt)))}


def tree_cp(tree, p, q, param=0, mode=TT):
    """Tiled critical path (units nb^3/3) of a tree on p x q tiles."""
    return int(_L().orc_tree_cp(_tree_id(tree), p, q, param, mode))


def coarse(p, q, elist):
    """Coarse-grain ASAP execution of a list: (cp, p x q step array)."""
    lib = _L()
    a = np.array(elist, dtype=np.int32).reshape(-1, 3).T.copy()
    out = np.zeros(p * q, dtype=np.int32)
    cp = lib.orc_coarse(p, q, len(elist), _p32(a[0]), _p32(a[1]), _p32(a[2]), _p32(out))
    return int(cp), out.reshape(p, q)


def fibonacci_coarse(p, q):
    """The thesis's Fibonacci time-step formula, p x q array."""
    out = np.zeros(p * q, dtype=np.int32)
    _L().orc_fib_coarse(p, q, _p32(out))
    return out.reshape(p, q)
