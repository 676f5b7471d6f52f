"""Brute-force dense references used to pin the oracle (test code only).

Independent of the oracle's implementation: these routines work on a dense copy
of the whole matrix and follow the textbook statement of each step.
"""
import numpy as np


def dense_step1(K, node_ptr, tau, dtype=np.float64, first_unit=True):
    """Per-block max-|diag| symmetric elimination with threshold postponing, dense.

    K: dense scaled matrix in elimination order.  The Schur complement of all
    indices still alive is kept explicitly; each accepted pivot is eliminated by
    one rank-1 update (eq. (2)); postponed indices are deleted (no further updates).
    Returns (pivot_sequence, D, postponed (sorted)).
    """
    n = K.shape[0]
    S = np.array(K, dtype=dtype)
    alive = np.ones(n, dtype=bool)
    seq, D, post = [], [], []
    for j in range(len(node_ptr) - 1):
        cand = list(range(int(node_ptr[j]), int(node_ptr[j + 1])))
        dprev, have = 1.0, first_unit
        while cand:
            vals = np.abs(np.array([S[k, k] for k in cand], dtype=np.float64))
            best = vals.max()
            k0 = min(k for k, v in zip(cand, vals) if v == best)
            d = S[k0, k0]
            if d == 0 or (have and abs(float(d)) < tau * abs(dprev)):
                post += cand
                alive[cand] = False
                break
            alive[k0] = False
            others = np.nonzero(alive)[0]
            col = S[others, k0].copy()
            row = S[k0, others].copy()
            S[np.ix_(others, others)] -= np.outer(col / d, row).astype(dtype)
            cand.remove(k0)
            seq.append(k0)
            D.append(float(d))
            dprev, have = float(d), True
    return np.array(seq), np.array(D), np.array(sorted(post), dtype=np.int64)


def dense_schur(K, l2):
    """S22 = K22 - K21 K11^{-1} K12 by LAPACK (numpy.linalg.solve)."""
    n = K.shape[0]
    l1 = np.setdiff1d(np.arange(n), l2)
    K11 = K[np.ix_(l1, l1)]
    K12 = K[np.ix_(l1, l2)]
    K22 = K[np.ix_(l2, l2)]
    return K22 - K12.T @ np.linalg.solve(K11, K12)


def svd_rank_deficiency(A, rel=1e-10):
    s = np.linalg.svd(A, compute_uv=False)
    return int(np.sum(s <= rel * s.max()))
