"""Python binding of the C ABI in include/hf.h (ctypes; argument marshalling only).

Every computation runs in the HIP library ``libhyfact.so`` built in-tree by
``paper_2208_01907_amd/build.py``.  PyTorch provides device memory and the HIP
stream.  If the library is missing this module raises at import time: there is
no fallback.

The function names follow the C entry points:

    ctx = hf_analyse(indptr, indices, perm, node_ptr, parent, opt)
    perm, node_ptr, parent = hf_order(indptr, indices)   # nested dissection of a pattern
    hf_factorize(ctx, values_dev)            # values: torch float64 on the GPU
    X = hf_solve(ctx, B_dev)                 # B: (L, r) torch float64 on the GPU
    k = hf_kernel_dim(ctx)
    N = hf_kernel_basis(ctx)                 # (L, k)
    lam2, S22 = hf_schur(ctx)                # hard part, Schur complement (scaled)
    q = hf_scaling(ctx)
    info = hf_info(ctx)
    piv = hf_pivots(ctx)                     # step-1 pivots, postponing margins
    mags = hf_s22_pivots(ctx)                # pivot magnitudes of the LDL^T of S22
    runs, nfac = hf_gcr_history(ctx)         # block-GCR residual histories
    Lam, GV = hf_adjoint(ctx, X, G)          # derivatives of a loss through X
    Y = hf_precond(ctx, R)                   # the preconditioner Q^{-1} (scaled, permuted)
    X = solve(ctx, values, B)                # torch.autograd-aware factorize + solve
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch first: it ships a HIP runtime under the same soname as the system one
# the library links; whichever loads first serves the process, and torch's own
# device initialisation fails when it is handed the other one
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libhyfact.so")

HF_OK = 0
HF_ERR_ARG = -1
HF_ERR_PATTERN = -2
HF_ERR_VALUE = -3
HF_ERR_STATE = -4
HF_ERR_NO_CONVERGENCE = -5
HF_ERR_BREAKDOWN = -6
HF_ERR_OOM = -7
HF_ERR_HIP = -8
HF_ERR_NOT_IMPLEMENTED = -9
HF_PREC_FP16 = 16
HF_PREC_FP16_PAIR = 17
HF_PREC_FP32 = 32
HF_PREC_FP64 = 64

EXPORTS = ["hf_default_options", "hf_analyse", "hf_factorize", "hf_solve", "hf_kernel_dim",
           "hf_kernel_basis", "hf_schur", "hf_scaling", "hf_info", "hf_strerror", "hf_destroy",
           "hf_timing_enable", "hf_timing_get", "hf_adjoint", "hf_pivots", "hf_s22_pivots", "hf_gcr_history",
           "hf_schur_noalloc", "hf_precond", "hf_order", "hf_tune"]

# kernel classes of hf_timing_get
KCLASS = ["panel", "permute_l11", "f11_update", "gather_border", "trsm", "syrk", "extend_add", "fwd_diag",
          "fwd_update", "bwd_border", "bwd_diag", "bwd_update", "solve_gather", "spmm", "gram", "combine",
          "other", "value_grad", "fwd_front", "bwd_front"]


class HFError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"{where}: {hf_strerror(code)} ({code})")


class HFOptions(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("low_precision", ctypes.c_int32),
                ("first_pivot_unit", ctypes.c_int32), ("n_enlarge", ctypes.c_int32),
                ("gcr_block", ctypes.c_int32), ("gcr_tol", ctypes.c_double),
                ("gcr_maxit", ctypes.c_int32), ("ker_tol", ctypes.c_double),
                ("refine_steps", ctypes.c_int32), ("refine_tol", ctypes.c_double),
                ("nd_leaf_max", ctypes.c_int32), ("sweep_front_min", ctypes.c_int32),
                ("sweep_wide_min", ctypes.c_int32),
                ("sweep_node_inverse", ctypes.c_int32)]


class HFInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_nodes", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("max_front", ctypes.c_int32), ("max_pivots", ctypes.c_int32),
                ("factor_entries", ctypes.c_int64), ("factor_flops", ctypes.c_double),
                ("factor_flops_done", ctypes.c_double), ("front_bytes", ctypes.c_int64),
                ("M", ctypes.c_int32), ("kernel_dim", ctypes.c_int32), ("gcr_blocks", ctypes.c_int32),
                ("gcr_iters_max", ctypes.c_int32), ("gcr_iters_total", ctypes.c_int32),
                ("solve_gcr_iters", ctypes.c_int32), ("rank_gap", ctypes.c_double),
                ("rank_candidates", ctypes.c_int32), ("state", ctypes.c_int32),
                ("t_analyse_ms", ctypes.c_double), ("t_step1_ms", ctypes.c_double),
                ("t_gcr_ms", ctypes.c_double), ("t_s22_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double)]


class HFKStat(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("launches", ctypes.c_int64), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double)]


def _load():
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is missing: build it with `python paper_2208_01907_amd/build.py` "
                          "(the HIP library is required; there is no fallback)")
    lib = ctypes.CDLL(LIBPATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "hf_default_options": (None, [P]),
        "hf_analyse": (ctypes.c_int, [I64, P, P, P, I32, P, P, P, P]),
        "hf_factorize": (ctypes.c_int, [P, P, P]),
        "hf_solve": (ctypes.c_int, [P, I32, P, I64, P, I64, P]),
        "hf_adjoint": (ctypes.c_int, [P, I32, P, I64, P, I64, P, I64, P, P]),
        "hf_kernel_dim": (ctypes.c_int, [P, P]),
        "hf_kernel_basis": (ctypes.c_int, [P, P, I64, P]),
        "hf_schur": (ctypes.c_int, [P, P, P, P, I64, P]),
        "hf_scaling": (ctypes.c_int, [P, P, P]),
        "hf_info": (ctypes.c_int, [P, P]),
        "hf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "hf_destroy": (None, [P]),
        "hf_timing_enable": (ctypes.c_int, [P, I32]),
        "hf_timing_get": (ctypes.c_int, [P, I32, P]),
        "hf_pivots": (ctypes.c_int, [P, P, P, P, P]),
        "hf_s22_pivots": (ctypes.c_int, [P, P]),
        "hf_gcr_history": (ctypes.c_int, [P, P, P, P, P]),
        "hf_schur_noalloc": (ctypes.c_int, [P, P, P, P, I64, P]),
        "hf_precond": (ctypes.c_int, [P, I32, P, P, P]),
        "hf_order": (ctypes.c_int, [I64, P, P, I32, P, P, P, P]),
        "hf_tune": (ctypes.c_int, [P, I32, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def hf_strerror(code: int) -> str:
    return _lib.hf_strerror(int(code)).decode()


def _check(code, where):
    if code != HF_OK:
        raise HFError(code, where)


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def hf_default_options(**kw) -> HFOptions:
    o = HFOptions()
    _lib.hf_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class Context:
    """Owns an hf_ctx; destroyed with the object."""

    def __init__(self, handle, n, nnz=0):
        self._h = handle
        self.n = n
        self.nnz = nnz
        self.generation = 0     # bumped by every successful hf_factorize

    @property
    def handle(self):
        if not self._h:
            raise ValueError("context destroyed")
        return self._h

    def destroy(self):
        if self._h:
            _lib.hf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def hf_order(indptr, indices, leaf_max=512):
    """Nested-dissection ordering of a CSR pattern (see hf_order in include/hf.h).
    Returns (perm, node_ptr, parent) as hf_analyse takes them."""
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    n = len(indptr) - 1
    perm = np.zeros(max(n, 1), dtype=np.int32)
    node_ptr = np.zeros(n + 1, dtype=np.int32)
    parent = np.zeros(max(n, 1), dtype=np.int32)
    nn = ctypes.c_int32()
    _check(_lib.hf_order(n, _np_ptr(indptr), _np_ptr(indices), int(leaf_max), _np_ptr(perm), ctypes.byref(nn),
                         _np_ptr(node_ptr), _np_ptr(parent)), "hf_order")
    k = nn.value
    return perm[:n].copy(), node_ptr[:k + 1].copy(), parent[:k].copy()


def hf_analyse(indptr, indices, perm=None, node_ptr=None, parent=None, opt=None) -> Context:
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    n = len(indptr) - 1
    perm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    node_ptr = None if node_ptr is None else np.ascontiguousarray(node_ptr, dtype=np.int32)
    parent = None if parent is None else np.ascontiguousarray(parent, dtype=np.int32)
    n_nodes = 0 if parent is None else len(parent)
    h = ctypes.c_void_p()
    code = _lib.hf_analyse(n, _np_ptr(indptr), _np_ptr(indices), _np_ptr(perm), n_nodes, _np_ptr(node_ptr),
                           _np_ptr(parent), ctypes.byref(opt) if opt is not None else None, ctypes.byref(h))
    _check(code, "hf_analyse")
    return Context(h, n, len(indices))


def hf_factorize(ctx: Context, values, stream=None):
    assert values.is_cuda and values.dtype == torch.float64 and values.is_contiguous()
    _check(_lib.hf_factorize(ctx.handle, ctypes.c_void_p(values.data_ptr()), _stream(stream)), "hf_factorize")
    ctx.generation += 1


def hf_solve(ctx: Context, B, X=None, stream=None):
    """Solve for B of shape (L, r) (float64, GPU).  Returns X of shape (L, r)."""
    assert B.is_cuda and B.dtype == torch.float64
    one = B.dim() == 1
    if B.dim() not in (1, 2):
        raise ValueError("B must be (L,) or (L, r)")
    B2 = B.reshape(B.shape[0], 1) if one else B
    r = B2.shape[1]
    Bc = B2.t().contiguous()                # column-major (L x r) storage
    Xc = torch.empty_like(Bc)
    _check(_lib.hf_solve(ctx.handle, r, ctypes.c_void_p(Bc.data_ptr()), ctx.n, ctypes.c_void_p(Xc.data_ptr()),
                         ctx.n, _stream(stream)), "hf_solve")
    out = Xc.t()
    if X is not None:
        X.copy_(out.reshape(X.shape))
        return X
    return out[:, 0] if one else out


def hf_tune(ctx: Context, r, stream=None):
    """Autotune the sweeps' launch shapes for r columns on the current factors
    (see hf_tune in include/hf.h).  Returns (sweep_front_min, sweep_wide_min, ms)."""
    fm, wm, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(_lib.hf_tune(ctx.handle, int(r), ctypes.byref(fm), ctypes.byref(wm), ctypes.byref(ms), _stream(stream)),
           "hf_tune")
    return fm.value, wm.value, ms.value


def hf_precond(ctx: Context, R, stream=None):
    """Q^{-1} R (see hf_precond in include/hf.h): R of shape (L, r), r <= 64,
    float64 on the GPU, rows in elimination order of the scaled matrix."""
    assert R.is_cuda and R.dtype == torch.float64 and R.dim() == 2
    Rc = R.contiguous()
    Y = torch.empty_like(Rc)
    _check(_lib.hf_precond(ctx.handle, Rc.shape[1], ctypes.c_void_p(Rc.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                           _stream(stream)), "hf_precond")
    return Y


def hf_adjoint(ctx: Context, X, G, with_values=True, stream=None):
    """Adjoint solve on the current factors (see hf_adjoint in include/hf.h).

    X: the solution hf_solve returned, G = dl/dX, both (L, r) or (L,) float64 on
    the GPU.  Returns (Lam, GV): Lam = Kbar^+ P G of the shape of G, and GV of
    shape (nnz,) = dl/dvalues on the analysed pattern (None if not with_values).
    """
    assert X.is_cuda and G.is_cuda and X.dtype == torch.float64 and G.dtype == torch.float64
    if X.shape != G.shape or X.dim() not in (1, 2):
        raise ValueError("X and G must both be (L,) or (L, r)")
    one = X.dim() == 1
    X2 = X.reshape(-1, 1) if one else X
    G2 = G.reshape(-1, 1) if one else G
    r = X2.shape[1]
    Xc = X2.t().contiguous()
    Gc = G2.t().contiguous()
    Lc = torch.empty_like(Gc)
    GV = torch.empty(ctx.nnz, dtype=torch.float64, device=X.device) if with_values else None
    _check(_lib.hf_adjoint(ctx.handle, r, ctypes.c_void_p(Xc.data_ptr()), ctx.n, ctypes.c_void_p(Gc.data_ptr()),
                           ctx.n, ctypes.c_void_p(Lc.data_ptr()), ctx.n,
                           ctypes.c_void_p(GV.data_ptr()) if GV is not None else None, _stream(stream)),
           "hf_adjoint")
    Lam = Lc.t()
    return (Lam[:, 0] if one else Lam), GV


class _HybridSolve(torch.autograd.Function):
    """values, B -> X = Kbar(values)^+ B with the adjoint of hf_adjoint as backward."""

    @staticmethod
    def forward(fctx, values, B, ctx):
        hf_factorize(ctx, values.detach().contiguous())
        X = hf_solve(ctx, B.detach())
        fctx.ctx = ctx
        fctx.generation = ctx.generation
        fctx.save_for_backward(X)
        return X

    @staticmethod
    def backward(fctx, gX):
        ctx = fctx.ctx
        if ctx.generation != fctx.generation:
            raise RuntimeError("the context was factorized again after this solve; its adjoint needs the "
                               "factors the solve used")
        (X,) = fctx.saved_tensors
        Lam, GV = hf_adjoint(ctx, X, gX.contiguous(), with_values=fctx.needs_input_grad[0])
        return GV, (Lam if fctx.needs_input_grad[1] else None), None


def solve(ctx: Context, values, B):
    """Factorize with ``values`` and solve for ``B``, differentiable in both.

    Gradients: dl/dB = Kbar^+ P dl/dX (P: projector onto the range) and
    dl/dvalues[(i, j)] = -sum_c Lam[i, c] X[j, c]; the latter is exact along value
    perturbations that keep the kernel of Kbar.  The backward pass reuses the
    context's factors and raises if it was factorized again in between.
    """
    return _HybridSolve.apply(values, B, ctx)


def hf_kernel_dim(ctx: Context) -> int:
    k = ctypes.c_int32()
    _check(_lib.hf_kernel_dim(ctx.handle, ctypes.byref(k)), "hf_kernel_dim")
    return k.value


def hf_kernel_basis(ctx: Context, stream=None):
    k = hf_kernel_dim(ctx)
    Nc = torch.zeros((k, ctx.n), dtype=torch.float64, device="cuda")
    if k:
        _check(_lib.hf_kernel_basis(ctx.handle, ctypes.c_void_p(Nc.data_ptr()), ctx.n, _stream(stream)),
               "hf_kernel_basis")
    return Nc.t()


def hf_schur(ctx: Context, stream=None):
    m = ctypes.c_int32()
    _check(_lib.hf_schur(ctx.handle, ctypes.byref(m), None, None, 0, _stream(stream)), "hf_schur")
    M = m.value
    lam = np.zeros(max(M, 1), dtype=np.int32)
    S = torch.zeros((max(M, 1), max(M, 1)), dtype=torch.float64, device="cuda")
    if M:
        _check(_lib.hf_schur(ctx.handle, ctypes.byref(m), _np_ptr(lam), ctypes.c_void_p(S.data_ptr()), M,
                             _stream(stream)), "hf_schur")
    return lam[:M], S[:M, :M].t()


def hf_schur_noalloc(ctx: Context, S_out=None, stream=None):
    """hf_schur through the allocation-free entry point.  S_out (an (M, M) float64
    CUDA tensor, column-major storage: its transpose is returned) may be given
    so that the call itself allocates nothing; the Python side allocates it
    otherwise."""
    m = ctypes.c_int32()
    _check(_lib.hf_schur_noalloc(ctx.handle, ctypes.byref(m), None, None, 0, _stream(stream)), "hf_schur_noalloc")
    M = m.value
    lam = np.zeros(max(M, 1), dtype=np.int32)
    S = S_out if S_out is not None else torch.zeros((max(M, 1), max(M, 1)), dtype=torch.float64, device="cuda")
    if M:
        _check(_lib.hf_schur_noalloc(ctx.handle, ctypes.byref(m), _np_ptr(lam), ctypes.c_void_p(S.data_ptr()), M,
                                     _stream(stream)), "hf_schur_noalloc")
    return lam[:M], S[:M, :M].t()


def hf_scaling(ctx: Context, stream=None):
    q = torch.zeros(ctx.n, dtype=torch.float64, device="cuda")
    _check(_lib.hf_scaling(ctx.handle, ctypes.c_void_p(q.data_ptr()), _stream(stream)), "hf_scaling")
    return q


def hf_info(ctx: Context) -> dict:
    info = HFInfo()
    _check(_lib.hf_info(ctx.handle, ctypes.byref(info)), "hf_info")
    return {name: getattr(info, name) for name, _ in HFInfo._fields_}


def hf_pivots(ctx: Context) -> dict:
    """Step-1 pivot record: per-node accepted counts, the pivots (elimination
    positions), the candidate that stopped each node and the postponing margins."""
    n_nodes = int(hf_info(ctx)["n_nodes"])
    npiv = np.zeros(max(n_nodes, 1), dtype=np.int32)
    d = np.zeros(max(ctx.n, 1), dtype=np.float64)
    dstop = np.zeros(max(n_nodes, 1), dtype=np.float64)
    margin = np.zeros(max(n_nodes, 1), dtype=np.float64)
    _check(_lib.hf_pivots(ctx.handle, _np_ptr(npiv), _np_ptr(d), _np_ptr(dstop), _np_ptr(margin)), "hf_pivots")
    return {"npiv": npiv[:n_nodes], "d": d[:ctx.n], "dstop": dstop[:n_nodes], "margin": margin[:n_nodes]}


def hf_s22_pivots(ctx: Context) -> np.ndarray:
    M = int(hf_info(ctx)["M"])
    mags = np.zeros(max(M, 1), dtype=np.float64)
    _check(_lib.hf_s22_pivots(ctx.handle, _np_ptr(mags)), "hf_s22_pivots")
    return mags[:M]


def hf_gcr_history(ctx: Context):
    """Residual histories of the block-GCR runs: (list of arrays, number of runs of hf_factorize)."""
    nr, nf = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.hf_gcr_history(ctx.handle, ctypes.byref(nr), ctypes.byref(nf), None, None), "hf_gcr_history")
    ptr = np.zeros(nr.value + 1, dtype=np.int32)
    _check(_lib.hf_gcr_history(ctx.handle, ctypes.byref(nr), None, _np_ptr(ptr), None), "hf_gcr_history")
    hist = np.zeros(max(int(ptr[-1]), 1), dtype=np.float64)
    _check(_lib.hf_gcr_history(ctx.handle, ctypes.byref(nr), None, None, _np_ptr(hist)), "hf_gcr_history")
    return [hist[ptr[r]:ptr[r + 1]].copy() for r in range(nr.value)], nf.value


def hf_timing_enable(ctx: Context, on: bool = True):
    _check(_lib.hf_timing_enable(ctx.handle, 1 if on else 0), "hf_timing_enable")


def hf_timing_get(ctx: Context) -> dict:
    out = {}
    for cls, name in enumerate(KCLASS):
        st = HFKStat()
        _check(_lib.hf_timing_get(ctx.handle, cls, ctypes.byref(st)), "hf_timing_get")
        out[name] = {"ms": st.ms, "launches": st.launches, "bytes": st.bytes, "flops": st.flops}
    return out
