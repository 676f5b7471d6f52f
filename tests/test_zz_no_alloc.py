"""Allocation-free Schur-complement accessor (hf_schur_noalloc) against hf_schur.

Two calls in a row on one GPU, the second with a smaller hard part, each
compared with hf_schur on the same context: the hard-part list and S22 must be
identical (both are exact permutations of the same data).
"""
import ctypes

import numpy as np
import pytest

from paper_2208_01907_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hy = pytest.importorskip("paper_2208_01907_amd.hyfact")


def _ctx(W, prec=64):
    opt = hy.hf_default_options(tau=W.tau, low_precision=prec, gcr_block=W.gcr_block)
    ctx = hy.hf_analyse(W.indptr, W.indices, W.perm, W.node_ptr, W.parent, opt)
    hy.hf_factorize(ctx, torch.tensor(W.values, device="cuda"))
    return ctx


def _noalloc(ctx, M):
    """Call the C entry point directly with caller-owned buffers."""
    lam = np.full(max(M, 1), -1, dtype=np.int32)
    S = torch.full((max(M, 1), max(M, 1)), float("nan"), dtype=torch.float64, device="cuda")
    m = ctypes.c_int32()
    code = hy._lib.hf_schur_noalloc(ctx.handle, ctypes.byref(m), ctypes.c_void_p(lam.ctypes.data),
                                    ctypes.c_void_p(S.data_ptr()), max(M, 1),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert code == hy.HF_OK, hy.hf_strerror(code)
    assert m.value == M
    torch.cuda.synchronize()
    return lam[:M], S[:M, :M].t().cpu().numpy()


def test_schur_noalloc_matches_schur_two_calls():
    big = _ctx(w.elasticity(6, seed=8, leaf_max=27, r=3, tau=0.9, gcr_block=0))      # M = 141
    small = _ctx(w.neumann2d(20, 18, seed=13, leaf_max=30, r=1))                        # M of a few
    sizes = []
    for ctx in (big, small):
        lam_ref, S_ref = hy.hf_schur(ctx)
        M = len(lam_ref)
        sizes.append(M)
        lam, S = _noalloc(ctx, M)
        assert np.array_equal(lam, lam_ref)
        assert np.array_equal(S, S_ref.cpu().numpy())
        # the size query with NULL buffers
        m = ctypes.c_int32()
        assert hy._lib.hf_schur_noalloc(ctx.handle, ctypes.byref(m), None, None, 0, None) == hy.HF_OK
        assert m.value == M
    assert sizes[0] > 64 and 0 < sizes[1] < sizes[0]


def test_schur_noalloc_errors():
    W = w.neumann2d(12, 10, seed=3, leaf_max=20, r=1)
    opt = hy.hf_default_options(tau=W.tau)
    ctx = hy.hf_analyse(W.indptr, W.indices, W.perm, W.node_ptr, W.parent, opt)
    m = ctypes.c_int32()
    assert hy._lib.hf_schur_noalloc(ctx.handle, ctypes.byref(m), None, None, 0, None) == hy.HF_ERR_STATE
    assert hy._lib.hf_schur_noalloc(None, ctypes.byref(m), None, None, 0, None) == hy.HF_ERR_ARG
    hy.hf_factorize(ctx, torch.tensor(W.values, device="cuda"))
    lam_ref, _ = hy.hf_schur(ctx)
    M = len(lam_ref)
    S = torch.zeros((M, M), dtype=torch.float64, device="cuda")
    assert hy._lib.hf_schur_noalloc(ctx.handle, ctypes.byref(m), None, ctypes.c_void_p(S.data_ptr()), M - 1,
                                    None) == hy.HF_ERR_ARG
