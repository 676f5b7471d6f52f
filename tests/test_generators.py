"""Input generators: sizes, symmetry, closed-form kernels, nested-dissection validity."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2208_01907_amd import workloads as w

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _check_nd(W):
    """Separator property: every coupling joins a node to itself or to an ancestor."""
    K = W.csr()
    n = W.n
    iperm = np.empty(n, dtype=np.int64)
    iperm[W.perm] = np.arange(n)
    node_of = np.repeat(np.arange(W.n_nodes), np.diff(W.node_ptr))
    anc = [set() for _ in range(W.n_nodes)]
    for j in range(W.n_nodes):
        p = W.parent[j]
        while p >= 0:
            anc[j].add(int(p))
            p = W.parent[p]
    coo = K.tocoo()
    a = node_of[iperm[coo.row]]
    b = node_of[iperm[coo.col]]
    for x, y in set(zip(a.tolist(), b.tolist())):
        assert x == y or y in anc[x] or x in anc[y], (x, y)
    # postorder: parent after child, subtrees contiguous
    assert np.all((W.parent == -1) | (W.parent > np.arange(W.n_nodes)))


@pytest.mark.parametrize("cfg,nnz,n,nodes", [("c1", 4992, 1024, 31), ("c3", 3501153, 46875, 383)])
def test_config_sizes(cfg, nnz, n, nodes):
    W = w.CONFIGS[cfg]()
    assert W.n == n and W.nnz == nnz and W.n_nodes == nodes
    K = W.csr()
    assert abs(K - K.T).max() == 0.0
    assert np.sort(W.perm).tolist() == list(range(n))


@pytest.mark.slow
def test_config_c2_size():
    W = w.config_c2()
    assert W.n == 262144 and W.nnz == 1810432 and W.n_nodes == 1023
    assert np.diff(W.node_ptr).max() == 4096


def test_closed_form_kernels():
    W = w.config_c1()
    K = W.csr()
    assert np.abs(K @ np.ones(W.n)).max() < 1e-9 * abs(K).max()
    E = w.elasticity(4, seed=1, r=1)
    KE = E.csr()
    Z = w.rigid_modes(4)
    assert np.abs(KE @ Z).max() < 1e-9 * abs(KE).max()
    # six independent rigid modes and nothing else: exactly 6 zero eigenvalues
    ev = np.linalg.eigvalsh(KE.toarray())
    assert np.sum(ev < 1e-9 * ev.max()) == 6


def test_rhs_is_consistent():
    W = w.elasticity(3, seed=2, r=3)
    assert np.abs(W.kernel.T @ W.x_star).max() < 1e-12
    assert np.allclose(W.csr() @ W.x_star, W.b)


@pytest.mark.parametrize("maker", [lambda: w.config_c1(), lambda: w.neumann2d(17, 9, seed=3, leaf_max=10),
                                   lambda: w.inclusions3d(10, 3, seed=4, leaf_max=40, r=1),
                                   lambda: w.elasticity(4, seed=5, leaf_max=8, r=1)])
def test_nested_dissection_valid(maker):
    _check_nd(maker())


def test_fig1_block_pattern():
    """A 3-level dissection of a 7x7 grid couples exactly the index sets of Fig. 1."""
    perm, node_ptr, parent = w.grid_nested_dissection((7, 7), leaf_max=9)
    assert len(parent) == 7
    # map our postorder (4,5,2,6,7,3,1 in the figure's names) to the figure's numbering
    root = int(np.nonzero(parent == -1)[0][0])
    lvl2 = sorted(int(j) for j in np.nonzero(parent == root)[0])
    name = {root: 1, lvl2[0]: 2, lvl2[1]: 3}
    k = 4
    for s in lvl2:
        for c in sorted(int(j) for j in np.nonzero(parent == s)[0]):
            name[c] = k
            k += 1
    K = w.fv_laplacian(np.ones((7, 7)))
    iperm = np.empty(49, dtype=np.int64)
    iperm[perm] = np.arange(49)
    node_of = np.repeat(np.arange(7), np.diff(node_ptr))
    coo = K.tocoo()
    pairs = {tuple(sorted((name[int(node_of[iperm[r]])], name[int(node_of[iperm[c]])])))
             for r, c in zip(coo.row, coo.col)}
    off = {p for p in pairs if p[0] != p[1]}
    want = set()
    for line in open(os.path.join(GOLDEN, "fig1_nd_blocks.txt")):
        line = line.split("#")[0].strip()
        if line:
            a, b = map(int, line.split())
            want.add(tuple(sorted((a, b))))
    assert off == want
    assert {p for p in pairs if p[0] == p[1]} == {(i, i) for i in range(1, 8)}


def test_mac_stokes_structure():
    """MAC Stokes saddle point: sizes (32^3: 95,232 face velocities + 32,768
    pressures), symmetry, an explicitly stored zero pressure diagonal, the
    constant pressure as the only kernel direction and the inertia of a
    saddle point (as many negative eigenvalues as pressures minus one) on a
    small grid, and a valid nested dissection of the staggered unknowns."""
    ids, nv = w._mac_face_ids(32)
    assert nv == 95232
    K, nv4 = w.mac_stokes(10.0 ** np.random.default_rng(1).uniform(-2, 2, size=(4, 4, 4)))
    assert nv4 == 3 * 3 * 16 and K.shape[0] == nv4 + 64
    assert abs(K - K.T).max() == 0.0
    assert np.all(K.diagonal()[nv4:] == 0.0)
    assert all(i in K.indices[K.indptr[i]:K.indptr[i + 1]] for i in range(K.shape[0]))
    one = np.zeros(K.shape[0])
    one[nv4:] = 1.0
    assert np.abs(K @ one).max() == 0.0
    ev = np.linalg.eigvalsh(K.toarray())
    tol = 1e-10 * np.abs(ev).max()
    assert (np.abs(ev) <= tol).sum() == 1 and (ev < -tol).sum() == 63 and (ev > tol).sum() == nv4
    W = w.stokes_mac(8, seed=4, leaf_max=64, r=2)
    _check_nd(W)
    assert sorted(W.perm.tolist()) == list(range(W.n))


def test_mac_viscosity_jacobian():
    """values(mu) = v0 + J mu entry by entry (A is linear in the viscosity, the
    divergence entries +-1/h do not depend on it)."""
    n = 4
    mu = 10.0 ** np.random.default_rng(2).uniform(-2, 2, size=(n, n, n))
    K, nv = w.mac_stokes(mu)
    J, v0 = w.mac_viscosity_jacobian(n)
    vals = v0 + J @ mu.reshape(-1, order="F")
    assert np.allclose(vals, K.data, rtol=1e-14, atol=0)
    assert set(np.abs(v0[v0 != 0.0]).tolist()) == {float(n)}
