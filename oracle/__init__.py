"""ORACLE -- test infrastructure, not part of the product.

A plain, slow CPU implementation of the hybrid factorization of Suzuki,
"A Hybrid Factorization Algorithm for Sparse Matrix with Mixed Precision
Arithmetic" (arXiv 2208.01907).  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with
the GPU library: its low-precision step 1 and preconditioner are plain C loops
(``hfo_step1.c``), everything else is NumPy/SciPy in FP64.

Where the paper is silent or ambiguous, the reading taken is stated in the
docstring of the function concerned; all of them are listed in the design notes.

Pipeline (Algorithm 1 and Algorithm 2 of Sec. 3):
  scale            -- K = Q Kbar Q with unit / zero diagonal (Sec. 2)
  symbolic         -- border sets of the nested-dissection tree (Sec. 2.2)
  factor_low       -- step 1: low-precision LDL^T, max-|diag| symmetric
                      pivoting, threshold postponing (Sec. 2.1-2.2, C code)
  precond          -- Q^{-1}: cast, forward/backward substitution, cast back
  bgcr             -- Algorithm 5 (preconditioned block GCR)
  gcr              -- Algorithm 4 (single right-hand side), used as a pin
  schur            -- step 4: S22 = K22 - K21 X12
  ldlt_pivoted     -- step 5: FP64 LDL^T of S22 with symmetric pivoting,
                      1x1 / 2x2 blocks (Bunch-Parlett)
  rank_reveal      -- second-stage postponing, n_e enlargement, kernel dimension
  hybrid_factorize / hybrid_solve -- Algorithms 1 and 2 end to end
  adjoint_solve / value_gradient -- derivatives through the solve (an
                      extension: one more solve, then -lam x^T on the pattern)
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
import time

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libhfo.so")
_lib = None


def build(force=True):
    """Compile the C part of the oracle (plain gcc, OpenMP)."""
    src = os.path.join(_HERE, "hfo_step1.c")
    objs = []
    for real, suf in (("float", "f32"), ("double", "f64")):
        obj = os.path.join(_HERE, f"hfo_step1_{suf}.o")
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-std=c11", f"-DREAL={real}",
                               f"-DSUFFIX={suf}", "-c", src, "-o", obj])
        objs.append(obj)
    tmp = _LIBPATH + ".tmp"
    subprocess.check_call(["gcc", "-shared", "-fopenmp", "-o", tmp] + objs + ["-lm"])
    os.replace(tmp, _LIBPATH)
    for o in objs:
        os.remove(o)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            build()
        lib = ctypes.CDLL(_LIBPATH)
        P = ctypes.c_void_p
        for suf in ("f32", "f64"):
            fn = getattr(lib, f"hfo_factor_{suf}")
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int32, P, P, P, P, ctypes.c_double,
                           ctypes.c_int32, P, P, P, P, P, P, P, P, P]
            fn = getattr(lib, f"hfo_precond_{suf}")
            fn.restype = None
            fn.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, P, P, P, P, P, P, P,
                           ctypes.c_int32, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


# ----------------------------------------------------------------------------
# Sec. 2: diagonal scaling
# ----------------------------------------------------------------------------

def scale(Kbar):
    """Diagonal scaling of Sec. 2: Q_ii = 1/sqrt(|Kbar_ii|) when Kbar_ii != 0, else 1.

    K = Q Kbar Q.  Reading: the paper writes 1/sqrt(Kbar_ii) but requires diagonal
    entries in {-1, 0, 1}, so the magnitude is used, and the diagonal of K is set
    to sign(Kbar_ii) exactly (no rounding of q_i^2 Kbar_ii).  The zero test is exact.
    Returns (q, K) with K a CSR matrix with the pattern of Kbar.
    """
    Kbar = sp.csr_matrix(Kbar)
    d = Kbar.diagonal()
    q = np.ones(Kbar.shape[0])
    nz = d != 0
    q[nz] = 1.0 / np.sqrt(np.abs(d[nz]))
    K = Kbar.copy().tocoo()
    K.data = q[K.row] * K.data * q[K.col]
    on = K.row == K.col
    K.data[on] = np.sign(d[K.row[on]])
    K = K.tocsr()
    K.sort_indices()
    return q, K


def permute(K, perm):
    """K in elimination order: Kp[i, j] = K[perm[i], perm[j]]."""
    Kp = sp.csr_matrix(K)[perm][:, perm].tocsr()
    Kp.sort_indices()
    return Kp


# ----------------------------------------------------------------------------
# Sec. 2.2: nested-dissection tree, borders
# ----------------------------------------------------------------------------

def symbolic(Kp, node_ptr, parent):
    """Border of every node of the elimination tree (indices in elimination order).

    border_j = indices after node j's range that are coupled to Lambda_j, plus the
    borders of its children that lie after node j's range.  With a valid nested
    dissection these are exactly the ancestor indices coupled to the subtree.
    """
    n_nodes = len(parent)
    children = [[] for _ in range(n_nodes)]
    for j, pj in enumerate(parent):
        if pj >= 0:
            children[pj].append(j)
    indptr, indices = Kp.indptr, Kp.indices
    borders = []
    for j in range(n_nodes):
        s, e = int(node_ptr[j]), int(node_ptr[j + 1])
        parts = [indices[indptr[s]:indptr[e]]]
        parts += [borders[c] for c in children[j]]
        allc = np.concatenate(parts) if parts else np.zeros(0, np.int64)
        b = np.unique(allc[allc >= e]).astype(np.int32)
        borders.append(b)
    border_ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    border_ptr[1:] = np.cumsum([len(b) for b in borders])
    border = np.concatenate(borders).astype(np.int32) if n_nodes else np.zeros(0, np.int32)
    return border_ptr, border


# ----------------------------------------------------------------------------
# Algorithm 1, step 1 (low precision)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Step1:
    dtype: type
    n: int
    node_ptr: np.ndarray
    parent: np.ndarray
    border_ptr: np.ndarray
    border: np.ndarray
    lptr: np.ndarray
    L: np.ndarray
    d: np.ndarray
    piv_order: np.ndarray
    npiv: np.ndarray
    margin: np.ndarray
    dstop: np.ndarray        # per node: value of the candidate that stopped it (NaN: none)
    tiegap: np.ndarray       # per node: smallest relative lead of an accepted pivot over its rival
    lambda2: np.ndarray      # postponed indices, elimination order, ascending
    is_l2: np.ndarray        # uint8 mask over elimination-order indices

    @property
    def M(self):
        return len(self.lambda2)

    def pivot_sequence(self):
        """Global indices of the accepted pivots in elimination order (Pi_1)."""
        out = []
        for j in range(len(self.npiv)):
            s = self.node_ptr[j]
            out.append(self.piv_order[s:s + self.npiv[j]])
        return np.concatenate(out) if out else np.zeros(0, np.int32)

    def pivots(self):
        out = []
        for j in range(len(self.npiv)):
            s = self.node_ptr[j]
            out.append(self.d[s:s + self.npiv[j]])
        return np.concatenate(out) if out else np.zeros(0)


def factor_low(Kp, node_ptr, parent, tau, dtype=np.float32, first_ref_unit=True, exclude=None,
               borders=None):
    """Step 1 of Algorithm 1 in precision ``dtype`` (np.float32 or np.float64)."""
    lib = _load()
    n = Kp.shape[0]
    node_ptr = np.ascontiguousarray(node_ptr, dtype=np.int32)
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    if borders is None:
        borders = symbolic(Kp, node_ptr, parent)
    border_ptr, border = borders
    p = np.diff(node_ptr).astype(np.int64)
    b = np.diff(border_ptr).astype(np.int64)
    sizes = (p + b) * p
    lptr = np.zeros(len(p) + 1, dtype=np.int64)
    lptr[1:] = np.cumsum(sizes)
    dt = np.dtype(dtype)
    suf = "f32" if dt == np.float32 else "f64"
    L = np.zeros(max(int(lptr[-1]), 1), dtype=dt)
    d = np.zeros(max(n, 1), dtype=dt)
    piv_order = np.zeros(max(n, 1), dtype=np.int32)
    npiv = np.zeros(max(len(p), 1), dtype=np.int32)
    margin = np.zeros(max(len(p), 1), dtype=np.float64)
    dstop = np.zeros(max(len(p), 1), dtype=np.float64)
    tiegap = np.zeros(max(len(p), 1), dtype=np.float64)
    indptr = np.ascontiguousarray(Kp.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(Kp.indices, dtype=np.int32)
    vals = np.ascontiguousarray(Kp.data, dtype=np.float64)
    exc = None if exclude is None else np.ascontiguousarray(exclude, dtype=np.uint8)
    rc = getattr(lib, f"hfo_factor_{suf}")(
        n, _ptr(indptr), _ptr(indices), _ptr(vals), len(p), _ptr(node_ptr), _ptr(parent),
        _ptr(border_ptr), _ptr(border), float(tau), 1 if first_ref_unit else 0, _ptr(exc), _ptr(lptr),
        _ptr(L), _ptr(d), _ptr(piv_order), _ptr(npiv), _ptr(margin), _ptr(dstop), _ptr(tiegap))
    if rc != 0:
        raise RuntimeError(f"oracle step 1 failed (code {rc})")
    npiv = npiv[:len(p)]
    is_l2 = np.zeros(n, dtype=np.uint8)
    for j in range(len(p)):
        s, e = node_ptr[j], node_ptr[j + 1]
        is_l2[piv_order[s + npiv[j]:e]] = 1
    lambda2 = np.nonzero(is_l2)[0].astype(np.int32)
    return Step1(dtype=dt.type, n=n, node_ptr=node_ptr, parent=parent, border_ptr=border_ptr,
                 border=border, lptr=lptr, L=L, d=d[:n], piv_order=piv_order[:n], npiv=npiv,
                 margin=margin[:len(p)], dstop=dstop[:len(p)], tiegap=tiegap[:len(p)], lambda2=lambda2,
                 is_l2=is_l2)


def tested_values(f1: Step1, j):
    """Values compared by the ratio tests of node j, in test order: the accepted
    pivots, then the candidate that stopped the node (if any), with the indices
    of the accepted ones (-1 for the stopping candidate)."""
    s = int(f1.node_ptr[j])
    n = int(f1.npiv[j])
    vals = list(f1.d[s:s + n].astype(np.float64))
    idx = list(f1.piv_order[s:s + n])
    if not math.isnan(float(f1.dstop[j])):
        vals.append(float(f1.dstop[j]))
        idx.append(-1)
    return np.array(vals, dtype=np.float64), np.array(idx, dtype=np.int64)


def decided_nodes(f_lo: Step1, f_hi: Step1, tau, first_ref_unit=True, factor=4.0):
    """Nodes whose low-precision postponing decisions do not depend on rounding.

    The threshold test of Sec. 2.2 compares |v| (the next pivot candidate) with
    tau |ref| (the previous accepted pivot, or 1 for a node's first test).  A
    pivot that results from heavy cancellation (a near-kernel direction) is
    dominated by the rounding of the low-precision arithmetic, and so may be the
    outcome of the test that uses it.  The rounding error of every tested value
    is measured against the FP64 run ``f_hi`` of the same step 1: test i of node
    j compares v_i with ref_i in both runs (same position of the same node), and
    its error is e_i = ||v_lo| - |v_hi|| + tau ||ref_lo| - |ref_hi||.  The test
    is fixed when its distance from the threshold in the low-precision run,
    ||v_lo| - tau |ref_lo||, exceeds factor * e_i: another low-precision
    computation of the same values (a different summation order) may move each
    of them by about the same amount again, which factor = 4 covers with room.
    A node is decided when both runs accept the same number of pivots and all of
    its tests are fixed.  Returns (decided mask, worst error-to-distance ratio of
    every node's tests; +inf when the runs disagree).
    """
    nn = len(f_lo.npiv)
    dec = np.zeros(nn, dtype=bool)
    worst = np.zeros(nn)
    for j in range(nn):
        vl, _ = tested_values(f_lo, j)
        vh, _ = tested_values(f_hi, j)
        if f_lo.npiv[j] != f_hi.npiv[j] or len(vl) != len(vh):
            worst[j] = math.inf
            continue
        if len(vl) == 0:
            dec[j] = True
            continue
        al, ah = np.abs(vl), np.abs(vh)
        rl = np.concatenate([[1.0], al[:-1]])
        rh = np.concatenate([[1.0], ah[:-1]])
        if not first_ref_unit:        # the first pivot of a node is not tested
            al, ah, rl, rh = al[1:], ah[1:], rl[1:], rh[1:]
        live = al != 0.0              # a zero candidate stops without a test
        err = np.abs(al - ah) + tau * np.abs(rl - rh)
        dist = np.abs(al - tau * rl)
        with np.errstate(divide="ignore", invalid="ignore"):
            q = np.where(live, err / dist, 0.0)
        worst[j] = float(np.max(q)) if len(q) else 0.0
        dec[j] = bool(np.all(~live | (dist > factor * err)))
    return dec, worst


def precond(f1: Step1, R):
    """Q^{-1} R: the low-precision LDL^T solve of K11 (Sec. 3.2), R in elimination order.

    R is cast to the factor precision (round to nearest) and the result cast back
    to FP64; rows of the hard part are zero in the result.
    """
    lib = _load()
    R = np.asarray(R, dtype=np.float64)
    one = R.ndim == 1
    Rc = np.asfortranarray(R.reshape(f1.n, -1))
    Y = np.zeros_like(Rc, order="F")
    suf = "f32" if np.dtype(f1.dtype) == np.float32 else "f64"
    getattr(lib, f"hfo_precond_{suf}")(
        f1.n, len(f1.npiv), _ptr(f1.node_ptr), _ptr(f1.border_ptr), _ptr(f1.border), _ptr(f1.lptr),
        _ptr(f1.L), _ptr(f1.d), _ptr(f1.piv_order), _ptr(f1.npiv), _ptr(f1.is_l2), Rc.shape[1],
        _ptr(Rc), _ptr(Y))
    return Y[:, 0] if one else np.ascontiguousarray(Y)


# ----------------------------------------------------------------------------
# Sec. 3.3: preconditioned GCR (Algorithm 4) and block GCR (Algorithm 5)
# ----------------------------------------------------------------------------

def _chol_solve_deflated(Mm, rhs, rel_tol=1e-14):
    """Solve Mm a = rhs for the small SPSD Gram matrix Mm with a pivoted Cholesky.

    Reading (the paper assumes the Gram matrices are invertible): directions whose
    pivot falls to rel_tol * max(diag) or below are deflated and get coefficient 0.
    """
    m = Mm.shape[0]
    A = Mm.copy()
    piv = np.arange(m)
    dmax = max(float(np.max(np.diag(A))) if m else 0.0, 0.0)
    rank = 0
    Lc = np.zeros((m, m))
    for i in range(m):
        k = i + int(np.argmax(np.diag(A)[i:]))
        if A[k, k] <= rel_tol * dmax or A[k, k] <= 0.0:
            break
        # symmetric exchange i <-> k
        A[[i, k], :] = A[[k, i], :]
        A[:, [i, k]] = A[:, [k, i]]
        Lc[[i, k], :i] = Lc[[k, i], :i]
        piv[[i, k]] = piv[[k, i]]
        Lc[i, i] = math.sqrt(A[i, i])
        Lc[i + 1:, i] = A[i + 1:, i] / Lc[i, i]
        A[i + 1:, i + 1:] -= np.outer(Lc[i + 1:, i], Lc[i + 1:, i])
        rank += 1
    out = np.zeros((m,) + rhs.shape[1:])
    if rank:
        y = rhs[piv[:rank]]
        L11 = Lc[:rank, :rank]
        z = np.linalg.solve(L11, y)           # forward (library triangular solve)
        x = np.linalg.solve(L11.T, z)
        out[piv[:rank]] = x
    return out, rank


@dataclasses.dataclass
class GCRInfo:
    iterations: int
    converged: bool
    history: list          # max relative residual after each update (recurrence residual)
    Qv: list               # search directions A P_m (for the orthogonality pins)
    P: list
    deflated: int


def bgcr(apply_A, prec, B, tol=1e-15, maxit=50, keep=False):
    """Algorithm 5: right-preconditioned block GCR for A X = B (Sec. 3.4).

    Notation of the paper: M_n = Qv_n^T Qv_n, A_n = Qv_n^T R_n,
    X += P_n M_n^{-1} A_n, R -= Qv_n M_n^{-1} A_n; W = Q^{-1} R, Z = A W,
    B_mn = -Qv_m^T Z for every m <= n, P_{n+1} = W + sum_m P_m M_m^{-1} B_mn and
    Qv_{n+1} = Z + sum_m Qv_m M_m^{-1} B_mn.
    Readings: the numerator of beta uses q_m (the paper prints q_n; q_m is the
    standard GCR coefficient and the one that gives the stated orthogonality);
    the initial guess solves Q X0 = B as in Algorithm 4; stopping: every column
    with b_k != 0 has ||r_k||_2 <= tol ||b_k||_2 (recurrence residual).
    """
    B = np.asarray(B, dtype=np.float64)
    one = B.ndim == 1
    B = B.reshape(B.shape[0], -1)
    bn = np.linalg.norm(B, axis=0)
    active = bn > 0
    bn_safe = np.where(active, bn, 1.0)

    def relres(R):
        rr = np.linalg.norm(R, axis=0) / bn_safe
        return float(np.max(rr[active])) if active.any() else 0.0

    X = prec(B)
    R = B - apply_A(X)
    hist = [relres(R)]
    info = GCRInfo(0, hist[-1] <= tol, hist, [], [], 0)
    if info.converged:
        return (X[:, 0] if one else X), info
    W = prec(R)
    P = [W]
    Qv = [apply_A(W)]
    Mch = [Qv[0].T @ Qv[0]]
    for n in range(maxit):
        An = Qv[n].T @ R
        alpha, rank = _chol_solve_deflated(Mch[n], An)
        info.deflated = max(info.deflated, Mch[n].shape[0] - rank)
        X = X + P[n] @ alpha
        R = R - Qv[n] @ alpha
        hist.append(relres(R))
        info.iterations = n + 1
        if hist[-1] <= tol:
            info.converged = True
            break
        W = prec(R)
        Z = apply_A(W)
        Pn, Qn = W.copy(), Z.copy()
        for m in range(n + 1):
            Bmn = -(Qv[m].T @ Z)
            beta, _ = _chol_solve_deflated(Mch[m], Bmn)
            Pn += P[m] @ beta
            Qn += Qv[m] @ beta
        P.append(Pn)
        Qv.append(Qn)
        Mch.append(Qn.T @ Qn)
    if keep:
        info.P, info.Qv = P, Qv
    return (X[:, 0] if one else X), info


def gcr(apply_A, prec, b, tol=1e-15, maxit=50):
    """Algorithm 4: right-preconditioned GCR, single right-hand side, with q_n = A p_n."""
    b = np.asarray(b, dtype=np.float64)
    x = prec(b)
    r = b - apply_A(x)
    bn = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bn]
    if hist[-1] <= tol:
        return x, hist
    w = prec(r)
    p = [w]
    q = [apply_A(w)]
    for n in range(maxit):
        alpha = np.dot(r, q[n]) / np.dot(q[n], q[n])
        x = x + alpha * p[n]
        r = r - alpha * q[n]
        hist.append(np.linalg.norm(r) / bn)
        if hist[-1] <= tol:
            break
        w = prec(r)
        z = apply_A(w)
        pn, qn = w.copy(), z.copy()
        for m in range(n + 1):
            beta = -np.dot(z, q[m]) / np.dot(q[m], q[m])
            pn += beta * p[m]
            qn += beta * q[m]
        p.append(pn)
        q.append(qn)
    return x, hist


# ----------------------------------------------------------------------------
# Algorithm 1, step 5: FP64 LDL^T of S22 with symmetric pivoting (1x1 / 2x2)
# ----------------------------------------------------------------------------

BP_ALPHA = (1.0 + math.sqrt(17.0)) / 8.0


@dataclasses.dataclass
class LDLT:
    perm: np.ndarray     # P: row k of P S P^T is row perm[k] of S
    L: np.ndarray        # unit lower
    D: np.ndarray        # block diagonal (1x1 and 2x2 blocks)
    blocks: list         # (start, size) of every pivot block in elimination order
    mags: np.ndarray     # pivot magnitude of every position (|d| or min |eig| of its 2x2 block)


def ldlt_pivoted(S):
    """Symmetric indefinite LDL^T with complete (Bunch-Parlett) pivoting, FP64.

    The paper only says the pivoting of S22 may need 2x2 entries; the textbook
    Bunch-Parlett rule is taken: with alpha = (1+sqrt 17)/8, a 1x1 pivot on the
    largest diagonal entry (ties: smallest index) if it is at least alpha times
    the largest off-diagonal magnitude, else the 2x2 pivot on the off-diagonal
    entry of largest magnitude.  An exactly zero remainder ends with zero pivots.
    """
    S = np.array(S, dtype=np.float64)
    m = S.shape[0]
    A = S.copy()
    perm = np.arange(m)
    L = np.eye(m)
    D = np.zeros((m, m))
    blocks = []
    mags = np.zeros(m)

    def swap(i, k):
        if i == k:
            return
        A[[i, k], :] = A[[k, i], :]
        A[:, [i, k]] = A[:, [k, i]]
        L[[i, k], :i] = L[[k, i], :i]
        perm[[i, k]] = perm[[k, i]]

    i = 0
    while i < m:
        sub = A[i:, i:]
        dg = np.abs(np.diag(sub))
        kd = int(np.argmax(dg))
        gd = dg[kd]
        off = np.abs(sub - np.diag(np.diag(sub)))
        if sub.shape[0] > 1:
            ko = np.unravel_index(int(np.argmax(off)), off.shape)
            go = off[ko]
        else:
            go = 0.0
        if gd == 0.0 and go == 0.0:
            for t in range(i, m):
                blocks.append((t, 1))
            break
        if gd >= BP_ALPHA * go:
            swap(i, i + kd)
            d = A[i, i]
            D[i, i] = d
            l = A[i + 1:, i] / d
            A[i + 1:, i + 1:] -= np.outer(l, A[i, i + 1:])
            L[i + 1:, i] = l
            A[i + 1:, i] = 0.0
            A[i, i + 1:] = 0.0
            mags[i] = abs(d)
            blocks.append((i, 1))
            i += 1
        else:
            r, c = sorted((int(ko[0]), int(ko[1])))
            swap(i, i + r)
            swap(i + 1, i + c)
            E = A[i:i + 2, i:i + 2].copy()
            D[i:i + 2, i:i + 2] = E
            C = A[i + 2:, i:i + 2]
            Lc = np.linalg.solve(E, C.T).T
            A[i + 2:, i + 2:] -= Lc @ C.T
            L[i + 2:, i:i + 2] = Lc
            A[i + 2:, i:i + 2] = 0.0
            A[i:i + 2, i + 2:] = 0.0
            ev = np.abs(np.linalg.eigvalsh(E))
            mags[i] = mags[i + 1] = float(ev.min())
            blocks.append((i, 2))
            i += 2
    return LDLT(perm=perm, L=L, D=D, blocks=blocks, mags=mags)


@dataclasses.dataclass
class RankInfo:
    k: int
    t_postponed: int     # size of the second-stage postponed set
    candidates: int      # postponed set after the n_e enlargement
    gap: float           # smallest non-kernel candidate magnitude / largest kernel one


def rank_reveal(ld: LDLT, tau, n_enlarge=4, ker_tol=1e-10):
    """Kernel dimension of S22 (Sec. 2.2 second stage, Algorithm 1 step 5).

    The pivot magnitudes of the complete-pivoting LDL^T are visited in elimination
    order; as in step 1 the first one is compared with 1, the unit diagonal of the
    scaled matrix, and every later one with its predecessor: the second-stage
    postponing starts at the first pivot that is zero or smaller than tau times
    its reference.  The last n_enlarge accepted pivots are moved to the postponed
    candidates (the enlargement that keeps image entries to compare against).
    Among the candidates, the kernel consists of the trailing pivots whose
    magnitude is at most ker_tol (K has unit diagonal, so ker_tol is relative to
    its size).  A 2x2 block counts as one pivot: when the enlarged candidate set
    would begin at the second half of a block, it begins at the block's first
    half.  This decision rule is this implementation's own: the paper cites
    the kernel detection of Suzuki-Roux 2014 without describing it.
    """
    mags = ld.mags
    m = len(mags)
    if m == 0:
        return RankInfo(0, 0, 0, math.inf)
    t = m
    prev = 1.0
    for i in range(m):
        if mags[i] == 0.0 or mags[i] < tau * prev:
            t = i
            break
        prev = mags[i]
    postponed = m - t
    accepted = t
    e = min(n_enlarge, accepted) if postponed > 0 else 0
    start = t - e
    # a 2x2 pivot block is one pivot: the candidate set starts at a block boundary,
    # so the kernel count never takes half of a block
    if any(b0 + 1 == start for b0, bs in ld.blocks if bs == 2):
        start -= 1
    k = 0
    for i in range(m - 1, start - 1, -1):
        if mags[i] <= ker_tol:
            k += 1
        else:
            break
    nonker = mags[start:m - k]
    ker = mags[m - k:]
    gap = (float(nonker.min()) / max(float(ker.max()), 1e-300)) if (k and len(nonker)) else math.inf
    return RankInfo(k=k, t_postponed=postponed, candidates=m - start, gap=gap)


def kernel_of_ldlt(ld: LDLT, k):
    """Null-space basis of S22 from its LDL^T: P^T [-L11^{-T} L21^T; I_k]."""
    m = ld.L.shape[0]
    if k == 0:
        return np.zeros((m, 0))
    r = m - k
    L11 = ld.L[:r, :r]
    L21 = ld.L[r:, :r]
    top = -np.linalg.solve(L11.T, L21.T) if r else np.zeros((0, k))
    Z = np.vstack([top, np.eye(k)])
    out = np.zeros_like(Z)
    out[ld.perm] = Z
    return out


def ldlt_solve_partial(ld: LDLT, k, y):
    """x with S22 x = y restricted to the nonsingular part: the k kernel pivots get 0."""
    m = ld.L.shape[0]
    y = np.asarray(y, dtype=np.float64).reshape(m, -1)
    z = np.linalg.solve(ld.L, y[ld.perm])
    r = m - k
    w = np.zeros_like(z)
    if r:
        w[:r] = np.linalg.solve(ld.D[:r, :r], z[:r])
    x = np.linalg.solve(ld.L.T, w)
    out = np.zeros_like(x)
    out[ld.perm] = x
    return out


# ----------------------------------------------------------------------------
# Algorithms 1 and 2 end to end
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class HybridFactor:
    n: int
    q: np.ndarray
    perm: np.ndarray
    Kp: sp.csr_matrix
    step1: Step1
    lambda1_mask: np.ndarray
    X12: np.ndarray          # N x M in elimination order (rows of the hard part are 0)
    S22: np.ndarray
    ldl: LDLT
    rank: RankInfo
    kernel: np.ndarray       # L x k orthonormal basis in original variables
    gcr_block: int
    gcr_tol: float
    gcr_maxit: int
    gcr_iters: list
    Kbar: sp.csr_matrix = None   # the caller's matrix (residual correction of the solve)
    seconds: dict = None         # wall time of steps 1, 3 (block GCR) and 4-5 (S22, rank)

    @property
    def M(self):
        return self.step1.M

    @property
    def k(self):
        return self.rank.k


def _masked_ops(Kp, is_l2):
    keep = (is_l2 == 0).astype(np.float64)
    K11 = sp.diags(keep) @ Kp @ sp.diags(keep)
    K11 = K11.tocsr()

    def apply_A(X):
        return K11 @ X
    return apply_A


def hybrid_factorize(Kbar, perm, node_ptr, parent, tau=1e-2, low=np.float32, gcr_block=16,
                     gcr_tol=1e-15, gcr_maxit=50, n_enlarge=4, ker_tol=1e-10, first_ref_unit=True):
    """Algorithm 1: factorization with an internal iterative solver.

    1. step 1 in precision ``low`` -> Lambda_1, Pi_1, Lambda_2 (reading: Lambda_2 is
       the set of all indices postponed by the tree factorization; the second
       stage and the enlargement act on S22 in FP64, see rank_reveal);
    2. 2x2 blocking (masks over one matrix in elimination order);
    3. K11 X12 = K12 by Algorithm 5 in column blocks of width ``gcr_block``
       (0: all M columns at once), preconditioned by step 1;
    4. S22 = K22 - K21 X12 in FP64, symmetrized;
    5. FP64 pivoted LDL^T of S22 and its kernel.
    """
    t0 = time.perf_counter()
    q, K = scale(Kbar)
    Kp = permute(K, perm)
    n = Kp.shape[0]
    f1 = factor_low(Kp, node_ptr, parent, tau, dtype=low, first_ref_unit=first_ref_unit)
    t1 = time.perf_counter()
    l2 = f1.lambda2
    M = len(l2)
    apply_A = _masked_ops(Kp, f1.is_l2)

    def prec(R):
        return precond(f1, R)

    keep = (f1.is_l2 == 0)
    X12 = np.zeros((n, M))
    iters = []
    if M:
        K12 = Kp[:, l2].toarray()
        K12[~keep] = 0.0
        mb = M if gcr_block <= 0 else gcr_block
        for c0 in range(0, M, mb):
            Bblk = K12[:, c0:c0 + mb]
            Xb, info = bgcr(apply_A, prec, Bblk, tol=gcr_tol, maxit=gcr_maxit)
            if not info.converged:
                raise RuntimeError("block GCR did not converge")
            X12[:, c0:c0 + mb] = Xb
            iters.append(info.iterations)
    t2 = time.perf_counter()
    if M:
        W = -X12
        W[l2, np.arange(M)] = 1.0
        S22 = (Kp @ W)[l2]
        S22 = 0.5 * (S22 + S22.T)
    else:
        S22 = np.zeros((0, 0))
    ld = ldlt_pivoted(S22)
    rk = rank_reveal(ld, tau, n_enlarge=n_enlarge, ker_tol=ker_tol)
    N2 = kernel_of_ldlt(ld, rk.k)
    kern = np.zeros((n, rk.k))
    if rk.k:
        kern = -X12 @ N2
        kern[l2] = N2
        nb = np.zeros_like(kern)
        nb[perm] = kern                   # back to original ordering
        nb = q[:, None] * nb              # Kbar (Q n) = 0 when K n = 0
        kern, _ = np.linalg.qr(nb)
    t3 = time.perf_counter()
    return HybridFactor(n=n, q=q, perm=np.asarray(perm), Kp=Kp, step1=f1, lambda1_mask=keep, X12=X12,
                        S22=S22, ldl=ld, rank=rk, kernel=kern, gcr_block=gcr_block, gcr_tol=gcr_tol,
                        gcr_maxit=gcr_maxit, gcr_iters=iters, Kbar=sp.csr_matrix(Kbar),
                        seconds={"step1": t1 - t0, "gcr": t2 - t1, "s22": t3 - t2})


def _algorithm2(hf: HybridFactor, b, tol=None):
    """Algorithm 2 on scaled right-hand sides b in elimination order: returns x.

    y1 = Algorithm 5 on K11 y1 = b1 (to relative residual tol, default the
    factorization's gcr_tol); y2 = b2 - K21 y1; x2 solves S22 x2 = y2 with 0 on
    the kernel pivots; x1 = y1 - X12 x2.
    """
    f1 = hf.step1
    l2 = f1.lambda2
    b1 = b.copy()
    b1[l2] = 0.0
    apply_A = _masked_ops(hf.Kp, f1.is_l2)
    y1, info = bgcr(apply_A, lambda R: precond(f1, R), b1, tol=hf.gcr_tol if tol is None else tol,
                    maxit=hf.gcr_maxit)
    y1 = y1.reshape(hf.n, -1)
    x = y1.copy()
    if len(l2):
        y2 = b[l2] - (hf.Kp @ y1)[l2]
        x2 = ldlt_solve_partial(hf.ldl, hf.k, y2)
        x = y1 - hf.X12 @ x2
        x[l2] = x2
    return x


def hybrid_solve(hf: HybridFactor, Bbar, refine_steps=1, Kbar=None, refine_tol=1e-3):
    """Algorithm 2, plus residual correction, with the minimum-norm choice for singular K.

    xbar = P(Q Pi^T Algorithm2(Pi Q bbar)) where P projects orthogonally to the
    detected kernel (reading for singular K: the minimum-norm solution); then
    refine_steps times xbar += P(Q Pi^T Algorithm2(Pi Q (bbar - Kbar xbar))).  The
    residual is taken in the caller's variables on the projected iterate: the
    scaled K has an exactly unit diagonal and differs from Q Kbar Q by rounding,
    and Kbar 1 is only zero up to rounding, so a large kernel component would
    pollute it.  The correction is not part of the paper's Algorithm 2; it is
    added for the 1e-14 backward-error target.  A correction only has to be
    accurate relative to the residual it corrects, so its block GCR stops at
    relative residual refine_tol.  The residual is accumulated in extended
    precision and rounded once: in FP64 its rounding error would be about
    eps |Kbar| |xbar|, as large as the residual of a backward-stable solution,
    and the correction could not reduce the forward error below cond * eps; with
    an accurate residual it converges to the solution of Kbar x = bbar itself
    (mixed-precision iterative refinement).  Kbar defaults to the matrix given
    to hybrid_factorize.
    """
    Bbar = np.asarray(Bbar, dtype=np.float64)
    one = Bbar.ndim == 1
    Bbar = Bbar.reshape(hf.n, -1)
    Kbar = hf.Kbar if Kbar is None else sp.csr_matrix(Kbar)

    def to_orig(xp):
        out = np.zeros_like(xp)
        out[hf.perm] = xp
        out = hf.q[:, None] * out
        if hf.k:
            out = out - hf.kernel @ (hf.kernel.T @ out)
        return out

    xbar = to_orig(_algorithm2(hf, (hf.q[:, None] * Bbar)[hf.perm]))
    Kl = Kbar.astype(np.longdouble) if refine_steps else None
    for _ in range(refine_steps):
        # residual in extended precision (x86 long double, 64-bit significand),
        # rounded to FP64 once
        rbar = np.asarray(Bbar.astype(np.longdouble) - Kl @ xbar.astype(np.longdouble), dtype=np.float64)
        xbar = xbar + to_orig(_algorithm2(hf, (hf.q[:, None] * rbar)[hf.perm], tol=refine_tol))
    return xbar[:, 0] if one else xbar


def backward_error(Kbar, X, B):
    """max over columns of ||b - K x||_inf / (||K||_inf ||x||_inf + ||b||_inf).

    The residual is accumulated in extended precision (x86 long double) so the
    check adds no error of its own at the 1e-14 level.
    """
    Kbar = sp.csr_matrix(Kbar)
    X = np.asarray(X, dtype=np.float64).reshape(Kbar.shape[0], -1)
    B = np.asarray(B, dtype=np.float64).reshape(Kbar.shape[0], -1)
    normK = float(np.max(np.asarray(abs(Kbar).sum(axis=1)).ravel()))
    rows = np.repeat(np.arange(Kbar.shape[0]), np.diff(Kbar.indptr))
    v = Kbar.data.astype(np.longdouble)
    worst = 0.0
    for c in range(X.shape[1]):
        prod = v * X[Kbar.indices, c].astype(np.longdouble)
        kx = np.zeros(Kbar.shape[0], dtype=np.longdouble)
        np.add.at(kx, rows, prod)
        r = B[:, c].astype(np.longdouble) - kx
        den = normK * np.max(np.abs(X[:, c])) + np.max(np.abs(B[:, c]))
        be = float(np.max(np.abs(r))) / den if den > 0 else 0.0
        worst = max(worst, be)
    return worst


# ----------------------------------------------------------------------------
# Adjoint of the solve (an extension of Algorithm 2, not a step of the paper)
# ----------------------------------------------------------------------------
# x = Kbar^+ b for b in the range of Kbar.  When Kbar moves along perturbations
# that keep its kernel, differentiating Kbar x = b gives dx = -Kbar^+ dKbar x, so a
# loss l(x) with g = dl/dx has dl/db = Kbar^+ P g and dl/dKbar_ij = -lam_i x_j with
# lam = Kbar^+ P g (P: orthogonal projector onto the range).

def adjoint_solve(Kbar, G, kernel):
    """lam = Kbar^+ P G, dense, for small matrices.

    With an orthonormal kernel basis N of the symmetric Kbar, Kbar + N N^T is
    non-singular and its inverse is Kbar^+ + N N^T; applied to P G (orthogonal to
    N) it gives Kbar^+ P G.  ``kernel`` may have zero columns (non-singular Kbar).
    """
    A = Kbar.toarray() if sp.issparse(Kbar) else np.array(Kbar, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    N = np.asarray(kernel, dtype=np.float64).reshape(A.shape[0], -1)
    PG = G - N @ (N.T @ G) if N.shape[1] else G
    return np.linalg.solve(A + N @ N.T, PG)


def value_gradient(indptr, indices, X, Lam):
    """dl/dvalues on a CSR pattern: entry (i, j) gets -sum_c Lam[i, c] X[j, c]."""
    X = np.asarray(X, dtype=np.float64)
    Lam = np.asarray(Lam, dtype=np.float64)
    X = X.reshape(X.shape[0], -1)
    Lam = Lam.reshape(Lam.shape[0], -1)
    rows = np.repeat(np.arange(len(indptr) - 1), np.diff(indptr))
    return -np.sum(Lam[rows] * X[np.asarray(indices)], axis=1)
