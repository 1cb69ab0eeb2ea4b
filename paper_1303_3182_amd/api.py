"""Tensor-level helpers over the C ABI (allocation and pointer marshalling
only; all arithmetic runs in libtqr.so)."""
import torch

from . import _binding as B


def _ptr(t):
    return None if t is None else ctypes_ptr(t)


def ctypes_ptr(t):
    return t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def colmajor(x, device="cuda"):
    """A column-major float64 device copy of a 2-D array/tensor (stride (1, m))."""
    t = torch.as_tensor(x, dtype=torch.float64)
    if t.dim() == 1:
        t = t[:, None]
    m, n = t.shape
    out = torch.empty((n, m), dtype=torch.float64, device=device).t()
    out.copy_(t)
    return out


def _ld(t):
    if t.dim() != 2 or t.stride(0) != 1 or t.dtype != torch.float64 or not t.is_cuda:
        raise B.TqrError("expected a column-major float64 CUDA tensor")
    return max(t.stride(1), t.shape[0])


def workspace(m, n, nrhs=0, opts=None, device="cuda"):
    nbytes = B.tqr_workspace_size(m, n, nrhs, opts)
    if nbytes == 0:
        raise B.TqrError("invalid shape/options for workspace")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def factor(A, opts=None, T=None, info=None, nrhs=0):
    """Factor the column-major tensor A in place; returns (A, T).  The
    workspace T is sized for a later apply_qt with up to nrhs columns."""
    m, n = A.shape
    if T is None:
        T = workspace(m, n, nrhs, opts, A.device)
    B.tqr_factor_ex(m, n, A.data_ptr(), _ld(A), T.data_ptr(), T.numel(), opts,
                    None if info is None else info.data_ptr(), _stream())
    return A, T


def apply_qt(A, T, Bm, opts=None, info=None):
    """B <- Q^T B for a factorization produced by factor() with the same opts."""
    m, n = A.shape
    B.tqr_apply_qt(m, n, A.data_ptr(), _ld(A), T.data_ptr(), T.numel(), Bm.shape[1], Bm.data_ptr(),
                   _ld(Bm), opts, None if info is None else info.data_ptr(), _stream())
    return Bm


def solve_r(A, T, Bm, opts=None, info=None):
    """B[:n] <- R^{-1} B[:n] with R from factor() (same opts)."""
    m, n = A.shape
    B.tqr_solve_r(m, n, A.data_ptr(), _ld(A), T.data_ptr(), T.numel(), Bm.shape[1], Bm.data_ptr(),
                  _ld(Bm), opts, None if info is None else info.data_ptr(), _stream())
    return Bm


def lstsq_workspace(m, n, nrhs=1, opts=None, device="cuda"):
    """Device workspace for lstsq (uint8 tensor of tqr_lstsq_work_size bytes)."""
    nbytes = B.tqr_lstsq_work_size(m, n, nrhs, opts)
    if nbytes == 0:
        raise B.TqrError("invalid shape/options for lstsq")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def lstsq(A, Bm, opts=None, X=None, work=None, info=None):
    """Least-squares solution X (n x nrhs) of min ||A X - B||; A, B untouched."""
    m, n = A.shape
    nrhs = Bm.shape[1]
    if X is None:
        X = torch.empty((nrhs, n), dtype=torch.float64, device=A.device).t()
    if work is None:
        work = lstsq_workspace(m, n, nrhs, opts, A.device)
    B.tqr_lstsq(m, n, nrhs, A.data_ptr(), _ld(A), Bm.data_ptr(), _ld(Bm), X.data_ptr(), _ld(X),
                work.data_ptr(), work.numel(), opts, None if info is None else info.data_ptr(), _stream())
    return X


def refine_report(work):
    """The refinement report that tqr_lstsq leaves at the start of its
    workspace: dict(done, iterations, backward_error, history)."""
    import numpy as np
    rec = 8 + 8 + 8 * B.REFINE_HISTORY + 8
    raw = work[:rec].cpu().numpy().tobytes()
    return _report(raw)


def _report(raw):
    import numpy as np
    done, iters = np.frombuffer(raw[:8], dtype=np.int32)
    vals = np.frombuffer(raw[8:8 + 8 + 8 * B.REFINE_HISTORY], dtype=np.float64)
    gm, ks = np.frombuffer(raw[16 + 8 * B.REFINE_HISTORY:24 + 8 * B.REFINE_HISTORY], dtype=np.int32)
    hist = [float(v) for v in vals[1:] if v >= 0.0]
    return {"done": int(done), "iterations": int(iters), "backward_error": float(vals[0]), "history": hist,
            "gmres_steps": int(gm), "krylov_steps": int(ks)}


def _i64arr(v):
    import ctypes
    return (ctypes.c_int64 * len(v))(*[int(x) for x in v])


def _ptrarr(ts):
    import ctypes
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


def lstsq_batched_workspace(shapes, nrhs=1, opts=None, device="cuda"):
    """Workspace for lstsq_batched over `shapes` [(m, n), ...]; opts.nb = 0
    sizes it for every built configuration (as the autotuner needs)."""
    ms = _i64arr([m for m, _ in shapes])
    ns = _i64arr([n for _, n in shapes])
    nbytes = B.lib().tqr_lstsq_batched_work_size(len(shapes), ms, ns, nrhs, B._opts_ptr(opts))
    if nbytes == 0:
        raise B.TqrError("invalid shapes/options for lstsq_batched")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _batch_args(As, Bs, Xs):
    ms = _i64arr([a.shape[0] for a in As])
    ns = _i64arr([a.shape[1] for a in As])
    return (ms, ns, _ptrarr(As), _i64arr([_ld(a) for a in As]), _ptrarr(Bs), _i64arr([_ld(b) for b in Bs]),
            _ptrarr(Xs), _i64arr([_ld(x) for x in Xs]))


def lstsq_batched(As, Bs, opts=None, Xs=None, work=None, info=None):
    """Least-squares solutions of a ragged batch in one executor launch.
    As[x]: m_x x n_x, Bs[x]: m_x x nrhs (column-major float64 CUDA tensors);
    returns the list of X[x] (n_x x nrhs)."""
    count = len(As)
    nrhs = Bs[0].shape[1]
    dev = As[0].device
    if Xs is None:
        Xs = [torch.empty((nrhs, a.shape[1]), dtype=torch.float64, device=dev).t() for a in As]
    if work is None:
        work = lstsq_batched_workspace([tuple(a.shape) for a in As], nrhs, opts, dev)
    ms, ns, pa, la, pb, lb, px, lx = _batch_args(As, Bs, Xs)
    rc = B.lib().tqr_lstsq_batched(count, ms, ns, nrhs, pa, la, pb, lb, px, lx, work.data_ptr(), work.numel(),
                                   B._opts_ptr(opts), None if info is None else info.data_ptr(), _stream())
    B._check(rc, "tqr_lstsq_batched")
    return Xs


def autotune_batched(As, Bs, opts, Xs=None, work=None):
    """Times every built (nb, ib) on this batch and sets opts.nb, opts.ib to
    the fastest; returns its time in ms (-1 if the choice was cached)."""
    import ctypes
    count = len(As)
    nrhs = Bs[0].shape[1]
    dev = As[0].device
    if Xs is None:
        Xs = [torch.empty((nrhs, a.shape[1]), dtype=torch.float64, device=dev).t() for a in As]
    if work is None:
        o0 = B.Opts()
        ctypes.memmove(ctypes.byref(o0), ctypes.byref(opts), ctypes.sizeof(B.Opts))
        o0.nb = 0
        work = lstsq_batched_workspace([tuple(a.shape) for a in As], nrhs, o0, dev)
    ms, ns, pa, la, pb, lb, px, lx = _batch_args(As, Bs, Xs)
    best = ctypes.c_float(0.0)
    rc = B.lib().tqr_autotune_batched(count, ms, ns, nrhs, pa, la, pb, lb, px, lx, work.data_ptr(), work.numel(),
                                      ctypes.byref(opts), ctypes.byref(best), _stream())
    B._check(rc, "tqr_autotune_batched")
    return best.value


def refine_reports(work, count):
    """The per-problem refinement reports at the start of a batched workspace."""
    import numpy as np
    rec = 8 + 8 + 8 * B.REFINE_HISTORY + 8
    raw = work[:rec * count].cpu().numpy().tobytes()
    return [_report(raw[rec * x:rec * (x + 1)]) for x in range(count)]


def cholinv(A, nb=64, variant=0, work=None, info=None):
    """In-place inverse of the SPD matrix whose lower triangle A holds
    (column-major float64 CUDA tensor): on return A's lower triangle holds
    that of A^{-1}.  variant: CHOLINV_INPLACE / CHOLINV_RENAMED (| CHOLINV_UUU)."""
    n = A.shape[0]
    if work is None:
        nbytes = B.tqr_cholinv_work_size(n, nb, variant)
        if nbytes == 0:
            raise B.TqrError("invalid size/options for cholinv")
        work = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    B.tqr_cholinv(n, A.data_ptr(), _ld(A), nb, variant, work.data_ptr(), work.numel(),
                  None if info is None else info.data_ptr(), _stream())
    return A


def zcolmajor(x, device="cuda"):
    """A column-major complex128 device copy of a 2-D array (stride (1, m))."""
    t = torch.as_tensor(x, dtype=torch.complex128)
    if t.dim() == 1:
        t = t[:, None]
    m, n = t.shape
    out = torch.empty((n, m), dtype=torch.complex128, device=device).t()
    out.copy_(t)
    return out


def _zld(t):
    if t.dim() != 2 or t.stride(0) != 1 or t.dtype != torch.complex128 or not t.is_cuda:
        raise B.TqrError("expected a column-major complex128 CUDA tensor")
    return max(t.stride(1), t.shape[0])


def zfactor(A, opts=None, W=None, info=None, nrhs=0):
    """Complex tiled QR of A in place; returns (A, W)."""
    m, n = A.shape
    if W is None:
        nbytes = B.tqr_zworkspace_size(m, n, nrhs, opts)
        if nbytes == 0:
            raise B.TqrError("invalid shape/options for zfactor")
        W = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    B.tqr_zfactor(m, n, A.data_ptr(), _zld(A), W.data_ptr(), W.numel(), opts,
                  None if info is None else info.data_ptr(), _stream())
    return A, W


def zapply_qh(A, W, Bm, opts=None, info=None):
    """B <- Q^H B for a factorization produced by zfactor with the same opts."""
    m, n = A.shape
    B.tqr_zapply_qh(m, n, A.data_ptr(), _zld(A), W.data_ptr(), W.numel(), Bm.shape[1], Bm.data_ptr(), _zld(Bm),
                    opts, None if info is None else info.data_ptr(), _stream())
    return Bm
