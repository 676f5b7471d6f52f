"""C ABI: the library loads and exports every entry point of include/hf.h; host-side
validation errors (returned before any device work, so they run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2208_01907_amd import hyfact as hy
from paper_2208_01907_amd import workloads as w

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "hf.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hf_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    names = _declared()
    assert "hf_analyse" in names and "hf_factorize" in names and "hf_solve" in names
    lib = ctypes.CDLL(hy.LIBPATH)
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(hy.EXPORTS) == names


def test_timing_classes_match_header():
    text = open(HEADER).read()
    enum = dict((k, int(v)) for k, v in re.findall(r"\b(HF_K_[A-Z0-9_]+)\s*=\s*(\d+)", text))
    assert enum["HF_K_NCLASS"] == len(hy.KCLASS)
    for i, name in enumerate(hy.KCLASS):
        assert enum["HF_K_" + name.upper()] == i


def test_strerror_and_defaults():
    assert hy.hf_strerror(0) == "ok"
    for code in range(-9, 0):
        assert hy.hf_strerror(code) not in ("ok", "unknown status")
    o = hy.hf_default_options()
    assert o.tau == 1e-2 and o.n_enlarge == 4 and o.low_precision == hy.HF_PREC_FP32
    assert o.gcr_tol == 1e-15 and o.gcr_block == 0 and o.refine_tol == 1e-3


def _analyse_code(indptr, indices, perm=None, node_ptr=None, parent=None, opt=None):
    try:
        hy.hf_analyse(indptr, indices, perm, node_ptr, parent, opt)
    except hy.HFError as e:
        return e.code
    return 0


def _small():
    W = w.neumann2d(5, 4, seed=1, leaf_max=6)
    return W


def test_pattern_errors():
    W = _small()
    ip, ix = W.indptr.copy(), W.indices.copy()
    bad = ix.copy()
    bad[ip[3]], bad[ip[3] + 1] = bad[ip[3] + 1], bad[ip[3]]      # unsorted row
    assert _analyse_code(ip, bad) == hy.HF_ERR_PATTERN
    bad = ix.copy()
    bad[0] = W.n + 5                                             # out of range
    assert _analyse_code(ip, bad) == hy.HF_ERR_PATTERN
    # drop one off-diagonal entry of row 0 -> unsymmetric pattern
    keep = np.ones(len(ix), bool)
    e = next(e for e in range(ip[0], ip[1]) if ix[e] != 0)
    keep[e] = False
    ip2 = ip.copy()
    ip2[1:] -= 1
    assert _analyse_code(ip2, ix[keep]) == hy.HF_ERR_PATTERN


def test_tree_and_option_errors():
    W = _small()
    ip, ix = W.indptr, W.indices
    perm = W.perm.copy()
    perm[0] = perm[1]                                            # not a permutation
    assert _analyse_code(ip, ix, perm, W.node_ptr, W.parent) == hy.HF_ERR_ARG
    par = W.parent.copy()
    par[0] = -1                                                  # breaks subtree contiguity / postorder
    if W.n_nodes > 2:
        assert _analyse_code(ip, ix, W.perm, W.node_ptr, par) in (hy.HF_ERR_ARG, hy.HF_ERR_PATTERN)
    # two leaves swapped under the wrong separators: couplings between sibling subtrees
    nodes = np.diff(W.node_ptr)
    rev = W.perm[::-1].copy()
    assert _analyse_code(ip, ix, rev, W.node_ptr, W.parent) == hy.HF_ERR_PATTERN
    o = hy.hf_default_options(tau=-1.0)
    assert _analyse_code(ip, ix, W.perm, W.node_ptr, W.parent, o) == hy.HF_ERR_ARG
    o = hy.hf_default_options(low_precision=8)
    assert _analyse_code(ip, ix, W.perm, W.node_ptr, W.parent, o) == hy.HF_ERR_ARG
    o = hy.hf_default_options(gcr_block=65)
    assert _analyse_code(ip, ix, W.perm, W.node_ptr, W.parent, o) == hy.HF_ERR_ARG


def test_size_limits():
    """A node of more than 4096 indices is refused before any device work."""
    n = 4097
    main = np.arange(n)
    rows = np.concatenate([main, main[:-1], main[1:]])
    cols = np.concatenate([main, main[1:], main[:-1]])
    K = __import__("scipy.sparse", fromlist=["csr_matrix"]).csr_matrix(
        (np.ones(len(rows)), (rows, cols)), shape=(n, n))
    K.sort_indices()
    perm, node_ptr, parent = w.single_node_tree(n)
    assert _analyse_code(K.indptr.astype(np.int64), K.indices.astype(np.int32), perm, node_ptr,
                         parent) == hy.HF_ERR_NOT_IMPLEMENTED


def test_diagnostics_reject_null_context():
    """hf_pivots, hf_s22_pivots, hf_gcr_history, hf_tune and hf_precond validate
    their arguments on the host (no device work)."""
    lib = hy._lib
    n = ctypes.c_int32()
    assert lib.hf_pivots(None, None, None, None, None) == hy.HF_ERR_ARG
    assert lib.hf_s22_pivots(None, None) == hy.HF_ERR_ARG
    assert lib.hf_gcr_history(None, ctypes.byref(n), None, None, None) == hy.HF_ERR_ARG
    assert lib.hf_tune(None, 16, None, None, None, None) == hy.HF_ERR_ARG
    assert lib.hf_precond(None, 16, None, None, None) == hy.HF_ERR_ARG


def test_node_above_4096_indices_is_refused():
    """The pivot block of a node lives in the registers of one workgroup (at most
    4096 rows).  A 65^3 grid has a root separator of 65^2 = 4225 indices:
    hf_analyse refuses it with HF_ERR_NOT_IMPLEMENTED before any device work,
    as it does a single-node matrix of more than 4096 indices (an ordering given
    without a tree; with neither, hf_analyse orders the pattern itself)."""
    W = w.inclusions3d(65, 0, seed=1, leaf_max=512, r=1)
    assert int(np.max(np.diff(W.node_ptr))) == 65 * 65
    assert _analyse_code(W.indptr, W.indices, W.perm, W.node_ptr, W.parent) == hy.HF_ERR_NOT_IMPLEMENTED
    n = 4097
    indptr = np.arange(n + 1, dtype=np.int64)
    indices = np.arange(n, dtype=np.int32)
    assert _analyse_code(indptr, indices, np.arange(n, dtype=np.int32)) == hy.HF_ERR_NOT_IMPLEMENTED
