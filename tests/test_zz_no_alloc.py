"""The allocation-free least-squares entry point (tqr_lstsq_noalloc, for
callers that cannot allocate device memory) against tqr_lstsq: the same
kernels and task graphs, so X and info must be identical bit for bit, on
two calls in a row (the second smaller, reusing the scratch array the first
left behind), in FP64 and with FP32 updates plus refinement.  Host-side
rejections (too large for the scratch array, the device-side selector)
enqueue nothing."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1303_3182_amd as T
import synth
from oracle import householder as H
from tests.gpu_util import EPS, case

pytestmark = pytest.mark.gpu


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _noalloc(A, Bm, opts):
    m, n = A.shape
    nrhs = Bm.shape[1]
    X = torch.full((nrhs, n), float("nan"), dtype=torch.float64, device="cuda").t()
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    rc = T.lib().tqr_lstsq_noalloc(m, n, nrhs, ctypes.c_void_p(A.data_ptr()), A.stride(1),
                                   ctypes.c_void_p(Bm.data_ptr()), Bm.stride(1), ctypes.c_void_p(X.data_ptr()),
                                   X.stride(1), ctypes.byref(opts), ctypes.c_void_p(info.data_ptr()), _stream())
    return rc, X, info


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_equals_lstsq_twice(dtype):
    for (m, n, nrhs, nb, seed) in [(1500, 700, 2, 128, 3), (700, 700, 1, 64, 4), (300, 100, 1, 64, 5)]:
        case("noalloc %s m=%d n=%d nrhs=%d nb=%d" % (dtype, m, n, nrhs, nb))
        A0 = synth.conditioned(n, 1e3, seed)[0] if m == n else synth.gaussian(m, n, seed)
        B0 = synth.gaussian_rhs(m, nrhs, seed)
        o = T.default_opts(nb=nb, tree="greedy", update_dtype=dtype, max_refine=20)
        A, Bm = T.colmajor(A0), T.colmajor(B0)
        rc, X, info = _noalloc(A, Bm, o)
        assert rc == 0, T.lib().tqr_strerror(rc)
        info_ref = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        Xr = T.lstsq(A, Bm, o, info=info_ref)
        torch.cuda.synchronize()
        assert int(info.item()) == int(info_ref.item()) == 0
        assert torch.equal(X, Xr)
        assert torch.equal(A, T.colmajor(A0)) and torch.equal(Bm, T.colmajor(B0))
        for c in range(nrhs):
            assert H.ls_backward_error(A0, B0[:, c], X[:, c].cpu().numpy()) <= 50 * EPS


def test_noalloc_host_rejections():
    case("noalloc rejections")
    big = T.default_opts(nb=256, tree="greedy")
    m, n = 8192, 2048  # A's copy alone is 128 MiB
    need = T.tqr_lstsq_work_size(m, n, 1, big)
    assert need > (64 << 20)
    A = torch.zeros((n, m), dtype=torch.float64, device="cuda").t()
    Bm = torch.zeros((1, m), dtype=torch.float64, device="cuda").t()
    rc, X, info = _noalloc(A, Bm, big)
    assert rc == -105  # TQR_E_SCRATCH
    assert b"scratch" in T.lib().tqr_strerror(rc)
    rc, X, info = _noalloc(A[:512, :256], Bm[:512], T.default_opts(tree="auto"))
    assert rc == -102  # TQR_E_UNSUPPORTED
    torch.cuda.synchronize()
    assert int(info.item()) == -7 and torch.isnan(X).all()  # nothing enqueued
