"""Pins of the oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a dense
brute-force elimination, LAPACK (Cholesky, solve, SVD, eigenvalues), closed-form
kernels, special cases that reduce to a textbook routine, or invariants the paper
states (orthogonality of GCR, Sec. 3.3).
"""
import math

import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2208_01907_amd import workloads as w
from tests import dense_ref


def _setup(W):
    q, K = oracle.scale(W.csr())
    Kp = oracle.permute(K, W.perm)
    return q, K, Kp


# --- Sec. 2: scaling -------------------------------------------------------

def test_scaling_identities():
    W = w.config_c1()
    Kbar = W.csr().tolil()
    Kbar[3, 3] = 0.0              # zero diagonal entry -> q = 1
    Kbar[5, 5] = -Kbar[5, 5]      # negative diagonal -> -1
    Kbar = Kbar.tocsr()
    q, K = oracle.scale(Kbar)
    d = K.diagonal()
    assert set(np.unique(d)) <= {-1.0, 0.0, 1.0}
    assert d[3] == 0.0 and d[5] == -1.0 and q[3] == 1.0
    coo = K.tocoo()
    off = coo.row != coo.col
    back = coo.data[off] / (q[coo.row[off]] * q[coo.col[off]])
    ref = np.asarray(Kbar[coo.row[off], coo.col[off]]).ravel()
    assert np.allclose(back, ref, rtol=4e-16, atol=0)


# --- Sec. 2.1-2.2: step 1 ---------------------------------------------------

@pytest.mark.parametrize("maker,tau,exact_order", [
    (lambda: w.neumann2d(8, 8, seed=11, leaf_max=9), 1e-2, True),
    (lambda: w.neumann2d(12, 7, seed=12, leaf_max=12, lo=-4, hi=4), 0.3, True),
    (lambda: w.inclusions3d(6, 2, seed=13, leaf_max=20, r=1), 1e-2, False),
    (lambda: w.elasticity(3, seed=14, leaf_max=8, r=1), 0.5, True),
    (lambda: w.random_dense_workload(30, seed=15, kernel_dim=2, indefinite=True), 0.1, True),
])
def test_step1_matches_dense_bruteforce(maker, tau, exact_order):
    """Same hard part and pivots as a dense elimination of the whole matrix.

    With a uniform coefficient (inclusions background) exact ties in exact
    arithmetic are broken by rounding, which differs between a dense in-place
    update and the tree's extend-add; there the pivot order inside a node may be
    a mirror image, so the per-node pivot multisets are compared instead.
    """
    W = maker()
    _, _, Kp = _setup(W)
    f1 = oracle.factor_low(Kp, W.node_ptr, W.parent, tau, dtype=np.float64)
    seq, D, post = dense_ref.dense_step1(Kp.toarray(), W.node_ptr, tau)
    assert np.array_equal(f1.lambda2, post)
    if exact_order:
        assert np.array_equal(f1.pivot_sequence(), seq)
        assert np.allclose(f1.pivots(), D, rtol=1e-10, atol=1e-14)
    node_of = np.repeat(np.arange(W.n_nodes), np.diff(W.node_ptr))
    got = f1.pivots()
    gseq = f1.pivot_sequence()
    for j in range(W.n_nodes):
        a = np.sort(got[node_of[gseq] == j])
        b = np.sort(D[node_of[seq] == j])
        assert np.allclose(a, b, rtol=1e-9, atol=1e-13)


def test_step1_fp32_matches_dense_fp32():
    W = w.neumann2d(10, 10, seed=16, leaf_max=16)
    _, _, Kp = _setup(W)
    f1 = oracle.factor_low(Kp, W.node_ptr, W.parent, W.tau, dtype=np.float32)
    seq, D, post = dense_ref.dense_step1(Kp.toarray(), W.node_ptr, W.tau, dtype=np.float32)
    assert np.array_equal(f1.lambda2, post)
    assert np.allclose(f1.pivots(), D, rtol=1e-4)


def test_step1_tau0_spd_is_cholesky():
    """tau = 0 on an SPD matrix: no postponing; L sqrt(D) is LAPACK's Cholesky factor."""
    W = w.neumann2d(9, 7, seed=17, leaf_max=10)
    K = W.csr() + sp.identity(W.n) * 1e-3 * abs(W.csr()).max()
    _, Ks = oracle.scale(K)
    Kp = oracle.permute(Ks, W.perm)
    f1 = oracle.factor_low(Kp, W.node_ptr, W.parent, 0.0, dtype=np.float64)
    assert f1.M == 0
    seq = f1.pivot_sequence()
    A = Kp.toarray()[np.ix_(seq, seq)]
    C = np.linalg.cholesky(A)
    D = f1.pivots()
    # rebuild L in pivot order from the dense LDL^T identity and compare
    Lr = C / np.sqrt(D)[None, :]
    assert np.allclose(Lr @ np.diag(D) @ Lr.T, A, atol=1e-12)
    assert np.allclose(np.diag(C) ** 2, D, rtol=1e-10)


def test_step1_spd_pivots_nonincreasing_in_each_node():
    W = w.inclusions3d(8, 3, seed=18, leaf_max=30, r=1)
    K = W.csr() + sp.identity(W.n) * 1e-2 * abs(W.csr()).max()
    _, Ks = oracle.scale(K)
    Kp = oracle.permute(Ks, W.perm)
    f1 = oracle.factor_low(Kp, W.node_ptr, W.parent, 0.0, dtype=np.float64)
    for j in range(W.n_nodes):
        s = W.node_ptr[j]
        d = f1.d[s:s + f1.npiv[j]]
        assert np.all(np.diff(d) <= 1e-12)


def test_step1_tau_above_one_postpones_everything():
    W = w.neumann2d(6, 5, seed=19, leaf_max=8)
    _, _, Kp = _setup(W)
    f1 = oracle.factor_low(Kp, W.node_ptr, W.parent, 2.0, dtype=np.float64)
    assert f1.M == W.n


# --- Sec. 3.2: preconditioner ------------------------------------------------

def test_precond_fp64_is_exact_inverse_of_k11():
    W = w.inclusions3d(7, 2, seed=20, leaf_max=25, r=1)
    _, _, Kp = _setup(W)
    f1 = oracle.factor_low(Kp, W.node_ptr, W.parent, W.tau, dtype=np.float64)
    l1 = np.nonzero(f1.is_l2 == 0)[0]
    rng = np.random.default_rng(0)
    R = np.zeros((W.n, 3))
    R[l1] = rng.standard_normal((len(l1), 3))
    Y = oracle.precond(f1, R)
    K11 = Kp.toarray()[np.ix_(l1, l1)]
    assert np.allclose(Y[l1], np.linalg.solve(K11, R[l1]), rtol=1e-9, atol=1e-12)
    assert np.all(Y[f1.lambda2] == 0.0)


# --- Sec. 3.3-3.4: GCR and block GCR -----------------------------------------

def _k11_problem(seed=21, low=np.float32):
    W = w.inclusions3d(8, 3, seed=seed, leaf_max=40, r=1)
    _, _, Kp = _setup(W)
    f1 = oracle.factor_low(Kp, W.node_ptr, W.parent, W.tau, dtype=low)
    keep = (f1.is_l2 == 0).astype(float)
    K11 = (sp.diags(keep) @ Kp @ sp.diags(keep)).tocsr()
    return W, Kp, f1, K11


def test_bgcr_solves_and_is_orthogonal():
    W, Kp, f1, K11 = _k11_problem()
    rng = np.random.default_rng(1)
    B = rng.standard_normal((W.n, 6))
    B[f1.lambda2] = 0.0
    X, info = oracle.bgcr(lambda V: K11 @ V, lambda R: oracle.precond(f1, R), B, tol=1e-15, keep=True)
    assert info.converged
    l1 = np.nonzero(f1.is_l2 == 0)[0]
    ref = np.linalg.solve(K11.toarray()[np.ix_(l1, l1)], B[l1])
    assert np.allclose(X[l1], ref, rtol=1e-10, atol=1e-12)
    # (A p_m, A p_n) = 0 for m != n (block form: Qv_m^T Qv_n = 0), Sec. 3.3 / 3.4
    Q = info.Qv
    for a in range(len(Q)):
        for b in range(a):
            G = Q[a].T @ Q[b]
            scale = np.linalg.norm(Q[a]) * np.linalg.norm(Q[b])
            assert np.abs(G).max() <= 1e-9 * scale


def test_block_gcr_with_one_column_is_gcr():
    """Algorithm 5 with a single right-hand side reproduces Algorithm 4."""
    W, Kp, f1, K11 = _k11_problem(seed=22)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(W.n)
    b[f1.lambda2] = 0.0
    A = lambda V: K11 @ V
    P = lambda R: oracle.precond(f1, R)
    x1, info = oracle.bgcr(A, P, b[:, None], tol=1e-15)
    x2, hist = oracle.gcr(A, P, b, tol=1e-15)
    assert info.iterations == len(hist) - 1
    assert np.allclose(info.history, hist, rtol=1e-6, atol=1e-17)
    assert np.allclose(x1[:, 0], x2, rtol=1e-12, atol=1e-14)


def test_bgcr_exact_preconditioner_stops_immediately():
    W, Kp, f1, K11 = _k11_problem(seed=23, low=np.float64)
    rng = np.random.default_rng(3)
    B = rng.standard_normal((W.n, 2))
    B[f1.lambda2] = 0.0
    _, info = oracle.bgcr(lambda V: K11 @ V, lambda R: oracle.precond(f1, R), B, tol=1e-13)
    assert info.iterations == 0


def test_bgcr_zero_and_dependent_columns():
    """Zero columns are excluded; a repeated column is deflated (the Gram matrix is singular)."""
    W, Kp, f1, K11 = _k11_problem(seed=24)
    rng = np.random.default_rng(4)
    B = rng.standard_normal((W.n, 4))
    B[f1.lambda2] = 0.0
    B[:, 2] = 0.0
    B[:, 3] = B[:, 0]
    X, info = oracle.bgcr(lambda V: K11 @ V, lambda R: oracle.precond(f1, R), B, tol=1e-14)
    assert info.converged
    assert np.all(X[:, 2] == 0.0)
    assert np.allclose(X[:, 3], X[:, 0], rtol=1e-10, atol=1e-13)


# --- Algorithm 1 steps 4-5 ----------------------------------------------------

def test_s22_matches_dense_schur():
    W = w.inclusions3d(8, 3, seed=25, leaf_max=40, r=1)
    hf = oracle.hybrid_factorize(W.csr(), W.perm, W.node_ptr, W.parent, tau=W.tau, gcr_block=2)
    assert hf.M > 0
    ref = dense_ref.dense_schur(hf.Kp.toarray(), hf.step1.lambda2)
    assert np.abs(hf.S22 - ref).max() <= 1e-11 * max(1.0, np.abs(hf.Kp).max())


def test_ldlt_pivoted_reconstructs_and_keeps_inertia():
    rng = np.random.default_rng(5)
    for n, indef in ((9, False), (11, True), (12, True)):
        V, _ = np.linalg.qr(rng.standard_normal((n, n)))
        s = rng.uniform(0.1, 2.0, n) * (rng.choice([-1, 1], n) if indef else 1)
        S = (V * s) @ V.T
        if indef:
            S[np.diag_indices(n)] = 0.0      # forces 2x2 pivots
        ld = oracle.ldlt_pivoted(S)
        P = np.eye(n)[ld.perm]
        assert np.allclose(ld.L @ ld.D @ ld.L.T, P @ S @ P.T, atol=1e-12)
        ev_d = np.concatenate([np.linalg.eigvalsh(ld.D[i:i + k, i:i + k]) for i, k in ld.blocks])
        ev_s = np.linalg.eigvalsh(S)
        assert (ev_d > 0).sum() == (ev_s > 0).sum()
        if indef:
            assert any(k == 2 for _, k in ld.blocks)


def test_kernel_count_never_splits_a_2x2_block():
    """Zero diagonal: only 2x2 pivots.  With n_enlarge = 3 the enlarged candidate
    set of the second stage would begin at the second half of a block; it begins
    at the block instead, so the kernel dimension counts whole blocks and equals
    the number of singular values at or below ker_tol (SVD)."""
    bv = [10.0 ** -i for i in range(10)] + [5e-11, 3e-11, 1e-16]
    W = w.paired_blocks_workload(bv, seed=50, n_tiny=3)
    sv = np.linalg.svd(W.csr().toarray(), compute_uv=False)
    for ne in (3, 4):
        hf = oracle.hybrid_factorize(W.csr(), W.perm, W.node_ptr, W.parent, tau=1e-2, gcr_block=0, n_enlarge=ne)
        assert hf.M == W.n and all(bs == 2 for _, bs in hf.ldl.blocks)
        assert hf.k == 6 == int((sv <= 1e-10).sum())
        assert (hf.M - hf.k) % 2 == 0                     # the rank cut is a block boundary
        X = oracle.hybrid_solve(hf, W.b)
        assert np.allclose(X, W.x_star, rtol=0, atol=1e-14 * np.abs(W.x_star).max())


def test_elasticity_cube_tau_rule():
    """The threshold of the 24^3 elastic cube follows its stated rule: at
    tau = 0.2 the FP32 and the FP64 step 1 both postpone exactly the six rigid
    modes (closed-form kernel dimension); at the grid value below (0.1) the FP32
    step 1 postpones fewer than six, so 0.2 is the smallest such grid value."""
    W = w.config_c3()
    assert W.tau == 0.2 and w.C3_TAU_GRID[w.C3_TAU_GRID.index(W.tau) - 1] == 0.1
    q, K = oracle.scale(W.csr())
    Kp = oracle.permute(K, W.perm)
    bd = oracle.symbolic(Kp, W.node_ptr, W.parent)
    f32 = oracle.factor_low(Kp, W.node_ptr, W.parent, 0.2, dtype=np.float32, borders=bd)
    f64 = oracle.factor_low(Kp, W.node_ptr, W.parent, 0.2, dtype=np.float64, borders=bd)
    assert f32.M == f64.M == 6
    assert oracle.factor_low(Kp, W.node_ptr, W.parent, 0.1, dtype=np.float32, borders=bd).M < 6


def test_batch_tau_rule():
    """The threshold of the 96-system batch follows its stated rule, recorded by
    tests/golden/make_c5_tau.py (oracle only): at the configured tau the FP32
    step 1 postpones at least one index of every system, at the grid value below
    at least one system postpones nothing.  Re-checked here with the oracle on the
    smallest system that fails at the grid value below."""
    path = os.path.join(os.path.dirname(__file__), "golden", "c5_tau.json")
    rec = json.load(open(path))
    tau = rec["tau"]
    grid = list(w.C3_TAU_GRID)
    below = grid[grid.index(tau) - 1]
    assert w.config_c5.__doc__ and f"{tau}" in w.config_c5.__doc__
    assert min(rec["M_fp32"][str(tau)]) >= 1 and min(rec["M_fp32"][str(below)]) == 0
    fails = [i for i, m in enumerate(rec["M_fp32"][str(below)]) if m == 0]
    i = min(fails, key=lambda i: rec["sides"][i])
    Wi = w.neumann3d(rec["sides"][i], seed=5000 + i, leaf_max=512, r=1)
    q, K = oracle.scale(Wi.csr())
    Kp = oracle.permute(K, Wi.perm)
    bd = oracle.symbolic(Kp, Wi.node_ptr, Wi.parent)
    assert oracle.factor_low(Kp, Wi.node_ptr, Wi.parent, below, dtype=np.float32, borders=bd).M == 0
    assert oracle.factor_low(Kp, Wi.node_ptr, Wi.parent, tau, dtype=np.float32, borders=bd).M >= 1


def test_decided_nodes_rule():
    """The rounding-independence rule: identical runs decide every node; a
    planted change of one tested value in the low-precision record (a near-tau
    pivot moved across the threshold) makes exactly that node undecided."""
    W = w.elasticity(5, seed=31, leaf_max=27, r=1, tau=0.3)
    q, K = oracle.scale(W.csr())
    Kp = oracle.permute(K, W.perm)
    f64 = oracle.factor_low(Kp, W.node_ptr, W.parent, W.tau, dtype=np.float64)
    dec, worst = oracle.decided_nodes(f64, f64, W.tau)
    assert dec.all() and np.all(worst == 0.0)
    f32 = oracle.factor_low(Kp, W.node_ptr, W.parent, W.tau, dtype=np.float32)
    dec32, worst32 = oracle.decided_nodes(f32, f64, W.tau)
    assert np.all(dec32 == ((f32.npiv == f64.npiv) & (worst32 < 0.25)))
    # move the second pivot of the last node to just above tau times the first
    j = len(W.parent) - 1
    s = f64.node_ptr[j]
    import copy
    g = copy.deepcopy(f64)
    g.d[s + 1] = np.float64(W.tau * abs(g.d[s]) * 1.001) * np.sign(g.d[s + 1])
    dec2, _ = oracle.decided_nodes(g, f64, W.tau)
    assert not dec2[j] and dec2[:j].all()


@pytest.mark.parametrize("kdim", [0, 1, 3])
def test_kernel_dimension_random_planted(kdim):
    W = w.random_dense_workload(24, seed=30 + kdim, kernel_dim=kdim, cond=1e3)
    hf = oracle.hybrid_factorize(W.csr(), W.perm, W.node_ptr, W.parent, tau=0.1, gcr_block=0)
    assert hf.k == kdim == dense_ref.svd_rank_deficiency(W.csr().toarray())


def test_kernel_dimension_closed_forms():
    W = w.config_c1()
    hf = oracle.hybrid_factorize(W.csr(), W.perm, W.node_ptr, W.parent, tau=W.tau, gcr_block=0)
    assert hf.k == 1
    # the detected kernel is the constant vector (principal angle ~ 0)
    c = np.ones(W.n) / math.sqrt(W.n)
    assert abs(abs(hf.kernel[:, 0] @ c) - 1.0) < 1e-8
    E = w.elasticity(5, seed=31, leaf_max=27, r=1)
    hfe = oracle.hybrid_factorize(E.csr(), E.perm, E.node_ptr, E.parent, tau=E.tau, gcr_block=8)
    assert hfe.k == 6
    Z, _ = np.linalg.qr(w.rigid_modes(5))
    s = np.linalg.svd(Z.T @ hfe.kernel, compute_uv=False)
    assert np.all(s > 1 - 1e-8)


# --- Algorithm 2 -------------------------------------------------------------

@pytest.mark.parametrize("low", [np.float32, np.float64])
def test_solve_is_minimum_norm_solution(low):
    W = w.neumann2d(10, 9, seed=32, leaf_max=12, r=2)
    hf = oracle.hybrid_factorize(W.csr(), W.perm, W.node_ptr, W.parent, tau=W.tau, low=low, gcr_block=0)
    X = oracle.hybrid_solve(hf, W.b)
    ref = np.linalg.pinv(W.csr().toarray()) @ W.b
    assert np.linalg.norm(X - ref) <= 1e-9 * np.linalg.norm(ref)
    assert oracle.backward_error(W.csr(), X, W.b) <= 1e-14


def test_solve_reaches_exact_solution_beyond_fp64_conditioning():
    """With the correction residual in extended precision the solve converges to
    the minimum-norm solution of the stored system itself, well below the
    cond * eps64 limit of an FP64 residual (the limit becomes cond * 2^-64 of the
    long-double residual).  Reference: dense LAPACK solves of Kbar + N N^T (N the
    orthonormal kernel), refined with residuals of Kbar x + N N^T x in long
    double (Kbar itself, not the rounded sum Kbar + N N^T).  Without the
    correction pass the error is larger."""
    W = w.neumann2d(16, 14, seed=34, lo=-4.0, hi=4.0, leaf_max=20, r=2)
    K = W.csr().toarray()
    N = W.kernel
    A = K + N @ N.T
    x = np.linalg.solve(A, W.b)
    Kl, Nl = K.astype(np.longdouble), N.astype(np.longdouble)
    for _ in range(5):
        xl = x.astype(np.longdouble)
        r = np.asarray(W.b.astype(np.longdouble) - Kl @ xl - Nl @ (Nl.T @ xl), dtype=np.float64)
        x = x + np.linalg.solve(A, r)
    cond = np.linalg.cond(A)
    limit64 = cond * 2.0 ** -52
    assert limit64 > 5e-9
    for low in (np.float32, np.float64):
        hf = oracle.hybrid_factorize(W.csr(), W.perm, W.node_ptr, W.parent, tau=W.tau, low=low, gcr_block=0)
        e1 = np.linalg.norm(oracle.hybrid_solve(hf, W.b) - x) / np.linalg.norm(x)
        e0 = np.linalg.norm(oracle.hybrid_solve(hf, W.b, refine_steps=0) - x) / np.linalg.norm(x)
        assert e1 <= 1e-3 * limit64 and e1 < e0


def test_solve_nonsingular_and_all_postponed():
    W = w.random_dense_workload(20, seed=33, kernel_dim=0, indefinite=True, cond=1e2, r=2)
    ref = np.linalg.solve(W.csr().toarray(), W.b)
    for tau in (1e-2, 2.0):   # tau > 1: everything postponed, S22 = K, plain pivoted LDL^T
        hf = oracle.hybrid_factorize(W.csr(), W.perm, W.node_ptr, W.parent, tau=tau, gcr_block=0)
        X = oracle.hybrid_solve(hf, W.b)
        assert np.allclose(X, ref, rtol=1e-9, atol=1e-12)
    assert hf.M == W.n


def test_backward_error_checker():
    W = w.config_c1()
    K = W.csr()
    assert oracle.backward_error(K, W.x_star, W.b) < 1e-15
    xp = W.x_star * (1 + 1e-10)
    be = oracle.backward_error(K, xp, W.b)
    assert 1e-13 < be < 1e-9


# --- adjoint of the solve (extension) ----------------------------------------
# Pins of oracle.adjoint_solve / oracle.value_gradient against central finite
# differences of solutions computed by LAPACK (numpy.linalg.solve / pinv).

def _loss(X, Xs):
    return 0.5 * float(np.sum((X - Xs) ** 2))


def test_adjoint_entrywise_finite_differences():
    """Non-singular K, each stored entry perturbed on its own (not symmetrically):
    dl/dK_ij = -lam_i x_j, which tells the entry (i, j) from (j, i)."""
    W = w.random_dense_workload(12, seed=40, kernel_dim=0, cond=10.0, r=2)
    A = W.csr().toarray()
    rng = np.random.default_rng(41)
    Xs = rng.standard_normal(W.b.shape)
    X = np.linalg.solve(A, W.b)
    lam = oracle.adjoint_solve(A, X - Xs, np.zeros((W.n, 0)))
    GV = oracle.value_gradient(W.indptr, W.indices, X, lam)
    rows = np.repeat(np.arange(W.n), np.diff(W.indptr))
    h = 1e-6
    fd = np.empty(W.nnz)
    for e in range(W.nnz):
        i, j = rows[e], W.indices[e]
        Ap, Am = A.copy(), A.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        fd[e] = (_loss(np.linalg.solve(Ap, W.b), Xs) - _loss(np.linalg.solve(Am, W.b), Xs)) / (2 * h)
    assert np.allclose(GV, fd, rtol=1e-6, atol=1e-8 * np.abs(fd).max())
    # a transposed formula (lam_j x_i) differs from the finite differences
    GVt = -np.sum(lam[W.indices] * X[rows], axis=1)
    assert not np.allclose(GVt, fd, rtol=1e-3, atol=1e-3 * np.abs(fd).max())


def test_adjoint_neumann_coefficient_directional_derivative():
    """Singular pure-Neumann FV operator: coefficient changes keep ker = constants,
    so l(c) = 1/2 ||Kbar(c)^+ B - X*||^2 is differentiable; the adjoint's
    directional derivatives in c and in B match finite differences of pinv."""
    rng = np.random.default_rng(42)
    coef = 10.0 ** rng.uniform(-1, 1, size=(6, 5))
    n = coef.size
    one = np.ones((n, 1)) / math.sqrt(n)
    B = rng.standard_normal((n, 3))
    B -= one @ (one.T @ B)
    Xs = rng.standard_normal((n, 3))
    K = w.fv_laplacian(coef)
    X = np.linalg.pinv(K.toarray()) @ B
    lam = oracle.adjoint_solve(K, X - Xs, one)
    GV = oracle.value_gradient(K.indptr, K.indices, X, lam)
    dc = coef * rng.uniform(-1, 1, size=coef.shape)
    h = 1e-6
    Kp, Km = w.fv_laplacian(coef + h * dc), w.fv_laplacian(coef - h * dc)
    assert np.array_equal(Kp.indices, K.indices) and np.array_equal(Km.indptr, K.indptr)
    dK = (Kp.data - Km.data) / (2 * h)
    fd = (_loss(np.linalg.pinv(Kp.toarray()) @ B, Xs) - _loss(np.linalg.pinv(Km.toarray()) @ B, Xs)) / (2 * h)
    assert abs(GV @ dK - fd) <= 1e-6 * abs(fd)
    dB = rng.standard_normal(B.shape)
    dB -= one @ (one.T @ dB)
    pinvK = np.linalg.pinv(K.toarray())
    fdb = (_loss(pinvK @ (B + h * dB), Xs) - _loss(pinvK @ (B - h * dB), Xs)) / (2 * h)
    assert abs(np.sum(lam * dB) - fdb) <= 1e-6 * abs(fdb)
    # kernel component of the loss gradient: projected away
    lam2 = oracle.adjoint_solve(K, X - Xs + 3.0 * one, one)
    assert np.allclose(lam2, lam, rtol=0, atol=1e-12 * np.abs(lam).max())
    assert np.abs(one.T @ lam).max() <= 1e-10 * np.abs(lam).max()


def test_adjoint_stokes_viscosity_gradient():
    """Enclosed MAC Stokes flow: the kernel (constant pressure) does not depend on
    the viscosity, so the gradient of l(mu) = 0.5 ||Kbar(mu)^+ b - x*||^2 (b made
    at a reference field, evaluated at another) is lam x^T on the pattern chained
    through d values / d mu.  Pinned by central differences (h = 1e-6) of
    solutions computed with LAPACK's pinv, along a seeded direction."""
    n = 3
    rng = np.random.default_rng(41)
    mu_ref = 10.0 ** rng.uniform(-2, 2, size=(n, n, n))
    mu = mu_ref * np.exp(rng.uniform(-0.5, 0.5, size=mu_ref.shape))
    K0, nv = w.mac_stokes(mu_ref)
    N = np.zeros((K0.shape[0], 1))
    N[nv:, 0] = 1.0 / np.sqrt(n ** 3)
    xs = rng.standard_normal((K0.shape[0], 2))
    xs -= N @ (N.T @ xs)
    b = K0 @ xs

    def loss(m):
        K, _ = w.mac_stokes(m)
        x = np.linalg.pinv(K.toarray()) @ b
        return 0.5 * float(np.sum((x - xs) ** 2))

    K, _ = w.mac_stokes(mu)
    x = oracle.adjoint_solve(K, b, N)
    lam = oracle.adjoint_solve(K, x - xs, N)
    gv = oracle.value_gradient(K.indptr, K.indices, x, lam)
    J, _ = w.mac_viscosity_jacobian(n)
    grad = J.T @ gv
    d = mu * rng.uniform(-1, 1, size=mu.shape)
    h = 1e-6
    fd = (loss(mu + h * d) - loss(mu - h * d)) / (2 * h)
    an = float(grad @ d.reshape(-1, order="F"))
    assert abs(an - fd) <= 1e-6 * abs(fd)


def test_bench_backward_error_matches_oracle():
    """The benchmark's backward-error measure (package metrics, SciPy's sparse
    product in long double) agrees with the oracle's (per-entry accumulation in
    long double) on exact, perturbed and zero solutions."""
    from paper_2208_01907_amd import metrics
    W = w.neumann2d(12, 9, seed=3, leaf_max=16, r=3)
    K = W.csr()
    rng = np.random.default_rng(8)
    X = np.linalg.lstsq(K.toarray(), W.b, rcond=None)[0]
    for Xt in (X, X + 1e-9 * rng.standard_normal(X.shape), np.zeros_like(X)):
        a, b = metrics.backward_error(K, Xt, W.b), oracle.backward_error(K, Xt, W.b)
        assert abs(a - b) <= 1e-3 * max(b, 1e-300) + 1e-20, (a, b)
