"""Accuracy measures reported by the benchmark (host side, NumPy/SciPy).

This is measurement code beside the product, not part of the method; the tests
check it against the oracle's own measure of the same quantity.
"""
import numpy as np
import scipy.sparse as sp


def backward_error(Kbar, X, B):
    """Normwise backward error max_c ||b - K x||_inf / (||K||_inf ||x||_inf + ||b||_inf).

    The product K x is formed by SciPy's sparse kernel in x86 extended precision
    (long double, 64-bit significand), so the measurement adds no error of its own
    at the 1e-14 level.
    """
    Kbar = sp.csr_matrix(Kbar)
    n = Kbar.shape[0]
    X = np.asarray(X, dtype=np.float64).reshape(n, -1)
    B = np.asarray(B, dtype=np.float64).reshape(n, -1)
    if n == 0:
        return 0.0
    normK = float(abs(Kbar).sum(axis=1).max())
    R = B.astype(np.longdouble) - Kbar.astype(np.longdouble) @ X.astype(np.longdouble)
    den = normK * np.abs(X).max(axis=0) + np.abs(B).max(axis=0)
    num = np.abs(R).max(axis=0).astype(np.float64)
    ok = den > 0
    return float((num[ok] / den[ok]).max()) if ok.any() else 0.0
