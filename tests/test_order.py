"""Nested-dissection ordering of general patterns (hf_order, host code).

Properties that make an ordering usable by the multifrontal factorization of
Sec. 2.2, checked on grids, a floating elastic body, random sparse patterns,
disconnected patterns and degenerate graphs: a permutation; nodes in postorder
with contiguous subtrees; every coupling between two nodes joins a node with an
ancestor (siblings' subtrees are separated); leaves within the size bound unless
a part is too shallow to split (a complete graph stays one node).  The ordering then drives the oracle's
factorization of a singular Neumann problem to its closed-form kernel."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2208_01907_amd import workloads as w

hy = pytest.importorskip("paper_2208_01907_amd.hyfact")


def _sym_pattern(K):
    K = sp.csr_matrix(K)
    P = ((abs(K) + abs(K.T)) + sp.eye(K.shape[0])).tocsr()
    P.sort_indices()
    return P


def check_ordering(P, perm, node_ptr, parent, leaf_max):
    n = P.shape[0]
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert node_ptr[0] == 0 and node_ptr[-1] == n and np.all(np.diff(node_ptr) > 0)
    nn = len(parent)
    assert len(node_ptr) == nn + 1
    first = np.arange(nn)
    nchild = np.zeros(nn, dtype=np.int64)
    for j in range(nn):
        pj = parent[j]
        assert pj == -1 or j < pj < nn
        if pj >= 0:
            first[pj] = min(first[pj], first[j])
            nchild[pj] += 1
    size = np.zeros(nn, dtype=np.int64)
    for j in range(nn):
        size[j] += 1
        if parent[j] >= 0:
            size[parent[j]] += size[j]
    assert np.all(size == np.arange(nn) - first + 1)   # subtrees contiguous in postorder
    node_of = np.empty(n, dtype=np.int64)
    for j in range(nn):
        node_of[perm[node_ptr[j]:node_ptr[j + 1]]] = j
    # every coupling joins a node with itself or an ancestor: with postorder,
    # node a is an ancestor of b iff first[a] <= b < a
    C = P.tocoo()
    a, b = node_of[C.row], node_of[C.col]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    assert np.all((lo == hi) | ((first[hi] <= lo) & (lo < hi)))
    leaves = np.nonzero(nchild == 0)[0]
    return int(np.diff(node_ptr)[leaves].max()), int(np.diff(node_ptr)[nchild > 0].max(initial=0))


PATTERNS = {
    "grid2d": lambda: w.neumann2d(40, 33, seed=1, r=1).csr(),
    "grid3d": lambda: w.inclusions3d(14, 3, seed=2, r=1).csr(),
    "elastic": lambda: w.elasticity(5, seed=3, r=1).csr(),
    "random": lambda: sp.random(3000, 3000, density=3.0 / 3000, random_state=np.random.RandomState(4)),
    "disconnected": lambda: sp.block_diag([w.neumann2d(20, 20, seed=5, r=1).csr(),
                                           w.inclusions3d(8, 1, seed=6, r=1).csr(),
                                           sp.eye(300)]),
    "path": lambda: sp.diags([np.ones(2999), np.ones(3000), np.ones(2999)], [-1, 0, 1]),
    "complete": lambda: sp.csr_matrix(np.ones((600, 600))),
    "star": lambda: sp.csr_matrix((np.ones(2 * 999), (np.r_[np.zeros(999), np.arange(1, 1000)],
                                                      np.r_[np.arange(1, 1000), np.zeros(999)])),
                                  shape=(1000, 1000)),
}


@pytest.mark.parametrize("name", list(PATTERNS))
@pytest.mark.parametrize("leaf", [64, 256])
def test_order_properties(name, leaf):
    P = _sym_pattern(PATTERNS[name]())
    perm, node_ptr, parent = hy.hf_order(P.indptr, P.indices, leaf)
    leaf_big, sep_big = check_ordering(P, perm, node_ptr, parent, leaf)
    again = hy.hf_order(P.indptr, P.indices, leaf)
    assert all(np.array_equal(x, y) for x, y in zip((perm, node_ptr, parent), again))   # deterministic
    if name == "complete":   # two levels from every start: too shallow to split
        assert len(parent) == 1
        return
    assert leaf_big <= leaf and len(parent) > 1
    if name == "star":   # the centre separates every leaf from every other
        assert sep_big == 1 and np.sum(parent == len(parent) - 1) == len(parent) - 1
    if name == "grid2d":
        assert sep_big <= 45          # a grid line (33 or 40) plus a few corner cells
    if name == "path":
        assert sep_big == 1


def test_order_empty_and_errors():
    perm, node_ptr, parent = hy.hf_order(np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32))
    assert len(perm) == 0 and list(node_ptr) == [0] and len(parent) == 0
    P = _sym_pattern(w.neumann2d(6, 5, seed=1, r=1).csr())
    with pytest.raises(hy.HFError) as e:
        hy.hf_order(P.indptr, P.indices, 0)
    assert e.value.code == hy.HF_ERR_ARG
    bad = P.indices.copy()
    bad[[0, 1]] = bad[[1, 0]]     # unsorted row
    with pytest.raises(hy.HFError) as e:
        hy.hf_order(P.indptr, bad, 16)
    assert e.value.code == hy.HF_ERR_PATTERN


def test_order_drives_the_oracle():
    """A coordinate-free ordering of a 3D Neumann problem: the oracle's hybrid
    factorization with it finds the closed-form kernel (constants) and solves to
    backward error 1e-14."""
    W = w.neumann3d(12, seed=8, r=2, leaf_max=64)
    perm, node_ptr, parent = hy.hf_order(W.indptr, W.indices, 64)
    hf = oracle.hybrid_factorize(W.csr(), perm, node_ptr, parent, tau=0.2, low=np.float64, gcr_block=0)
    assert hf.k == 1
    X = oracle.hybrid_solve(hf, W.b)
    assert oracle.backward_error(W.csr(), X, W.b) <= 1e-14


def test_order_splits_nodes_above_the_limit():
    """A 65^3 grid: its largest level-structure separator exceeds the 4096 indices
    a node may hold (the generator's axis-plane separator has 65^2 = 4225); the
    ordering splits such separators into chains of nodes of at most 4096, each
    the parent of the one before, and stays a valid dissection."""
    P = _sym_pattern(w.fv_laplacian(np.ones((65, 65, 65))))
    perm, node_ptr, parent = hy.hf_order(P.indptr, P.indices, 512)
    check_ordering(P, perm, node_ptr, parent, 512)
    sizes = np.diff(node_ptr)
    assert sizes.max() <= 4096
    chained = [j for j in range(len(parent) - 1) if parent[j] == j + 1 and sizes[j] + sizes[j + 1] > 4096
               and np.sum(parent == j) > 0]
    assert chained   # at least one separator was split into a chain
