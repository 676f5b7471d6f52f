"""Accuracy measures reported by the benchmark (host side, NumPy)."""
import numpy as np
import scipy.sparse as sp


def backward_error(Kbar, X, B):
    """Normwise backward error max_c ||b - K x||_inf / (||K||_inf ||x||_inf + ||b||_inf).

    The residual is accumulated in x86 extended precision (long double) so the
    measurement adds no error of its own at the 1e-14 level.
    """
    Kbar = sp.csr_matrix(Kbar)
    n = Kbar.shape[0]
    X = np.asarray(X, dtype=np.float64).reshape(n, -1)
    B = np.asarray(B, dtype=np.float64).reshape(n, -1)
    normK = float(np.max(np.asarray(abs(Kbar).sum(axis=1)).ravel())) if n else 0.0
    rows = np.repeat(np.arange(n), np.diff(Kbar.indptr))
    v = Kbar.data.astype(np.longdouble)
    worst = 0.0
    for c in range(X.shape[1]):
        kx = np.zeros(n, dtype=np.longdouble)
        np.add.at(kx, rows, v * X[Kbar.indices, c].astype(np.longdouble))
        r = B[:, c].astype(np.longdouble) - kx
        den = normK * np.max(np.abs(X[:, c])) + np.max(np.abs(B[:, c]))
        if den > 0:
            worst = max(worst, float(np.max(np.abs(r))) / den)
    return worst
