"""GPU tests of the adjoint of the solve (hf_adjoint and the autograd wrapper).

The adjoint is an extension of Algorithm 2: one more solve on the same factors
gives Lam = Kbar^+ P G for a loss gradient G = dl/dX (P projects onto the range),
and dl/dvalues[(i, j)] = -sum_c Lam[i, c] X[j, c] on the stored pattern.

Parity, against two references computed by the oracle alone:
- the oracle's hybrid method (oracle.hybrid_solve, oracle.value_gradient) for a G
  already in the range (projected with the closed-form kernel), and
- the oracle's dense pseudo-inverse solve (oracle.adjoint_solve) for a G with a
  kernel component (drawn from its own seed) that the projection must remove.
Bar: relative error <= max(1e-10, 4 x the dense solver's own forward error on X)
for Lam, twice that for the value gradient (a product of two such quantities),
and backward error <= 1e-14 of Lam against P G.  Unlike the solution X, whose
right-hand side is K x* with x* smooth, a random G excites the smallest
eigenvalues, and one correction pass (refine_steps = 1, as in hf_solve) leaves
both hybrid solves about cond(K) * eps apart: on the 14^3 inclusions (contrast
1e6) Lam agrees with the hybrid oracle to 2.5e-10 and with the dense one to
6e-10, inside the bar of 2.7e-9; the other cases agree to 1e-12 or better.  At the benchmark sizes the oracle's dense solve does not fit;
there the checks are properties that hold at any size: the backward error of Lam
and the identity sum(GV * values) = -trace(Lam^T B) for K X = B.  The backward
error bar there is looser (see the test): the projection uses the detected kernel,
whose distance to the closed form bounds how consistent P G is.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2208_01907_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hy = pytest.importorskip("paper_2208_01907_amd.hyfact")

CASES = {
    "c1": lambda: w.config_c1(),
    "inc14": lambda: w.inclusions3d(14, 4, seed=12, leaf_max=64, r=4, gcr_block=8),
    "n2d_ragged": lambda: w.neumann2d(67, 45, seed=7, leaf_max=100, r=2, gcr_block=8),
    "el6": lambda: w.elasticity(6, seed=8, leaf_max=27, r=5, gcr_block=8),
    "dense_k2": lambda: w.random_dense_workload(150, seed=10, kernel_dim=2, cond=1e3, r=3),
    "stokes8": lambda: w.stokes_mac(8, seed=4, leaf_max=64, r=4),
}


def _ctx(W, prec, gcr_block=None):
    opt = hy.hf_default_options(tau=W.tau, low_precision=prec,
                                gcr_block=W.gcr_block if gcr_block is None else gcr_block)
    return hy.hf_analyse(W.indptr, W.indices, W.perm, W.node_ptr, W.parent, opt)


def _loss_gradient(W, seed):
    """dl/dX drawn from its own seed, with a kernel component added."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal(W.b.shape)
    if W.kernel.shape[1]:
        G = G + W.kernel @ rng.standard_normal((W.kernel.shape[1], W.b.shape[1]))
    return G


def _project(W, G):
    N = W.kernel
    return G - N @ (N.T @ G) if N.shape[1] else G


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_parity(name, prec):
    W = CASES[name]()
    print(f"adjoint case {name} prec {prec} n={W.n} r={W.b.shape[1]}", flush=True)
    K = W.csr()
    G = _loss_gradient(W, 500)
    Xref = oracle.adjoint_solve(K, W.b, W.kernel)          # Kbar^+ B (B is in the range)
    Lref = oracle.adjoint_solve(K, G, W.kernel)
    GVref = oracle.value_gradient(W.indptr, W.indices, Xref, Lref)
    ctx = _ctx(W, prec)
    hy.hf_factorize(ctx, torch.tensor(W.values, device="cuda"))
    X = hy.hf_solve(ctx, torch.tensor(W.b, device="cuda"))
    Lam, GV = hy.hf_adjoint(ctx, X, torch.tensor(G, device="cuda"))
    Lam, GV = Lam.cpu().numpy(), GV.cpu().numpy()
    # the oracle's hybrid method, same precision of step 1 as the GPU run
    ref = oracle.hybrid_factorize(K, W.perm, W.node_ptr, W.parent, tau=W.tau,
                                  low=np.float32 if prec == 32 else np.float64, gcr_block=W.gcr_block,
                                  n_enlarge=W.meta.get("n_enlarge", 4))
    Gc = _project(W, G)
    Lc, GVc = hy.hf_adjoint(ctx, X, torch.tensor(Gc, device="cuda"))
    Xh, Lh = oracle.hybrid_solve(ref, W.b), oracle.hybrid_solve(ref, Gc)
    GVh = oracle.value_gradient(W.indptr, W.indices, Xh, Lh)
    rh = np.linalg.norm(Lc.cpu().numpy() - Lh) / np.linalg.norm(Lh)
    rgh = np.linalg.norm(GVc.cpu().numpy() - GVh) / np.linalg.norm(GVh)
    fwd = np.linalg.norm(Xref - W.x_star) / np.linalg.norm(W.x_star)
    bar = max(1e-10, 4 * fwd)
    rl = np.linalg.norm(Lam - Lref) / np.linalg.norm(Lref)
    rg = np.linalg.norm(GV - GVref) / np.linalg.norm(GVref)
    be = oracle.backward_error(K, Lam, _project(W, G))
    print(f"  vs hybrid oracle: rel(Lam)={rh:.2e} rel(GV)={rgh:.2e}; vs dense oracle: rel(Lam)={rl:.2e} "
          f"rel(GV)={rg:.2e} bar={bar:.1e}; be(Lam)={be:.2e}", flush=True)
    assert rh <= bar
    assert rgh <= 2 * bar
    assert rl <= bar
    assert rg <= 2 * bar
    assert be <= 1e-14
    if W.kernel.shape[1]:
        # orthogonal to the detected kernel, which agrees with the closed form to
        # about the same relative accuracy as the solutions
        assert np.linalg.norm(W.kernel.T @ Lam) <= bar * np.linalg.norm(Lam)


def _grid_problem(nx, ny, seed, leaf_max=64, r=2):
    rng = np.random.default_rng(seed)
    coef = 10.0 ** rng.uniform(-1, 1, size=(nx, ny))
    n = nx * ny
    one = np.ones((n, 1)) / math.sqrt(n)
    B = rng.standard_normal((n, r))
    B -= one @ (one.T @ B)
    Xs = rng.standard_normal((n, r))
    dc = coef * rng.uniform(-1, 1, size=coef.shape)
    dB = rng.standard_normal((n, r))
    dB -= one @ (one.T @ dB)
    return coef, B, Xs, dc, dB


@pytest.mark.parametrize("prec", [32, 64])
def test_autograd_matches_finite_differences(prec):
    """hyfact.solve through torch.autograd: directional derivatives in the
    per-cell coefficients (through the value gradient) and in B (through Lam)
    against central differences of the GPU solve itself."""
    nx, ny = 24, 20
    coef, B, Xs, dc, dB = _grid_problem(nx, ny, seed=13)
    perm, node_ptr, parent = w.grid_nested_dissection((nx, ny), 64)
    K = w.fv_laplacian(coef)
    opt = hy.hf_default_options(tau=1e-2, low_precision=prec, gcr_block=0)
    ctx = hy.hf_analyse(K.indptr, K.indices, perm, node_ptr, parent, opt)
    dev = "cuda"
    Xs_t = torch.tensor(Xs, device=dev)

    def loss(vals, Bm):
        X = hy.solve(ctx, torch.tensor(vals, device=dev), torch.tensor(Bm, device=dev))
        return 0.5 * float(((X - Xs_t) ** 2).sum())

    v = torch.tensor(K.data, device=dev, requires_grad=True)
    Bt = torch.tensor(B, device=dev, requires_grad=True)
    X = hy.solve(ctx, v, Bt)
    (0.5 * ((X - Xs_t) ** 2).sum()).backward()
    gv = v.grad.cpu().numpy()
    gb = Bt.grad.cpu().numpy()
    h = 1e-5
    Kp, Km = w.fv_laplacian(coef + h * dc), w.fv_laplacian(coef - h * dc)
    assert np.array_equal(Kp.indices, K.indices) and np.array_equal(Km.indptr, K.indptr)
    dK = (Kp.data - Km.data) / (2 * h)
    fd = (loss(Kp.data, B) - loss(Km.data, B)) / (2 * h)
    fdb = (loss(K.data, B + h * dB) - loss(K.data, B - h * dB)) / (2 * h)
    print(f"  prec {prec}: coef {gv @ dK:.10e} vs fd {fd:.10e}; B {np.sum(gb * dB):.10e} vs fd {fdb:.10e}",
          flush=True)
    assert abs(gv @ dK - fd) <= 1e-5 * abs(fd)
    assert abs(np.sum(gb * dB) - fdb) <= 1e-5 * abs(fdb)
    # the factors were replaced since X was computed: its backward must refuse
    X2 = hy.solve(ctx, torch.tensor(K.data, device=dev, requires_grad=True), torch.tensor(B, device=dev))
    hy.hf_factorize(ctx, torch.tensor(Kp.data, device=dev))
    with pytest.raises(RuntimeError):
        X2.sum().backward()


def test_adjoint_errors():
    W = w.config_c1()
    ctx = _ctx(W, 32)
    X = torch.zeros((W.n, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(hy.HFError) as e:
        hy.hf_adjoint(ctx, X, X.clone())
    assert e.value.code == hy.HF_ERR_STATE
    hy.hf_factorize(ctx, torch.tensor(W.values, device="cuda"))
    L = torch.empty(W.n, dtype=torch.float64, device="cuda")
    p = L.data_ptr()
    # Lam aliasing G is refused before any work
    assert hy._lib.hf_adjoint(ctx.handle, 1, X.data_ptr(), W.n, p, W.n, p, W.n, None, None) == hy.HF_ERR_ARG
    L2 = torch.empty(W.n, dtype=torch.float64, device="cuda")
    assert hy._lib.hf_adjoint(ctx.handle, 1, X.data_ptr(), W.n - 1, p, W.n, L2.data_ptr(), W.n,
                              None, None) == hy.HF_ERR_ARG
    # the value gradient aliasing X is refused
    assert hy._lib.hf_adjoint(ctx.handle, 1, X.data_ptr(), W.n, L2.data_ptr(), W.n, p, W.n, X.data_ptr(),
                              None) == hy.HF_ERR_ARG
    # r = 0: the value gradient is zero
    GV = torch.full((W.nnz,), 7.0, dtype=torch.float64, device="cuda")
    assert hy._lib.hf_adjoint(ctx.handle, 0, None, 0, None, 0, None, 0, GV.data_ptr(), None) == hy.HF_OK
    assert float(GV.abs().max()) == 0.0


@pytest.mark.parametrize("cfg", ["c2", "c3", "c4"])
def test_adjoint_full_size_properties(cfg):
    """Benchmark-size configurations (launch configuration of the benchmark): the
    backward error of Lam against P G and sum(GV * values) = -trace(Lam^T B)."""
    W = w.CONFIGS[cfg]()
    print(f"adjoint full size {cfg} n={W.n} r={W.b.shape[1]}", flush=True)
    G = _loss_gradient(W, 501)
    ctx = _ctx(W, 32, gcr_block=0)
    hy.hf_factorize(ctx, torch.tensor(W.values, device="cuda"))
    X = hy.hf_solve(ctx, torch.tensor(W.b, device="cuda"))
    Lam, GV = hy.hf_adjoint(ctx, X, torch.tensor(G, device="cuda"))
    Lam, GV = Lam.cpu().numpy(), GV.cpu().numpy()
    be = oracle.backward_error(W.csr(), Lam, _project(W, G))
    lhs = float(GV @ W.values)
    rhs = -float(np.sum(Lam * W.b))
    gap = abs(lhs - rhs) / (np.linalg.norm(Lam) * np.linalg.norm(W.b))
    ker = np.linalg.norm(W.kernel.T @ Lam) / np.linalg.norm(Lam)
    print(f"  be(Lam)={be:.2e} identity gap={gap:.2e} kernel component={ker:.2e}", flush=True)
    # the library projects G with the kernel basis it detected; at this size (1e6
    # contrast, 2.6e5 unknowns) that basis is 4.5e-8 from the closed form, and the
    # projected right-hand side is consistent only to that accuracy: Algorithm 2
    # returns the inconsistent part as a residual on the hard rows (measured
    # 8.8e-13; the same solve of an exactly consistent right-hand side reaches
    # 6e-15, see the solve tests)
    assert be <= 1e-11
    assert gap <= 1e-12
    assert ker <= 1e-7


def test_adjoint_many_rhs_chunked():
    """More right-hand sides than one block of the small dense kernels (64): the
    projection, the solve and the value gradient run in chunks."""
    W = w.config_c1()
    rng = np.random.default_rng(502)
    N = W.kernel
    Xs = rng.standard_normal((W.n, 70))
    Xs -= N @ (N.T @ Xs)
    B = W.csr() @ Xs
    G = rng.standard_normal((W.n, 70))
    Xref = oracle.adjoint_solve(W.csr(), B, N)
    Lref = oracle.adjoint_solve(W.csr(), G, N)
    GVref = oracle.value_gradient(W.indptr, W.indices, Xref, Lref)
    ctx = _ctx(W, 32)
    hy.hf_factorize(ctx, torch.tensor(W.values, device="cuda"))
    X = hy.hf_solve(ctx, torch.tensor(B, device="cuda"))
    Lam, GV = hy.hf_adjoint(ctx, X, torch.tensor(G, device="cuda"))
    rl = np.linalg.norm(Lam.cpu().numpy() - Lref) / np.linalg.norm(Lref)
    rg = np.linalg.norm(GV.cpu().numpy() - GVref) / np.linalg.norm(GVref)
    print(f"  70 RHS: rel(Lam)={rl:.2e} rel(GV)={rg:.2e}", flush=True)
    assert rl <= 1e-10 and rg <= 2e-10
    # without the value gradient: the same Lam (the same arithmetic), no GV
    Lam2, GV2 = hy.hf_adjoint(ctx, X, torch.tensor(G, device="cuda"), with_values=False)
    assert GV2 is None and torch.equal(Lam2, Lam)


def test_autograd_elasticity_moduli():
    """Floating Q1 elastic cube: the rigid modes stay the kernel for every modulus
    field, so the value gradient chained to per-element moduli matches central
    differences of the GPU solve (both directions drawn from their own seed)."""
    ne = 5
    rng = np.random.default_rng(14)
    young = 10.0 ** rng.uniform(0, 1, size=(ne, ne, ne))
    K = w.q1_elasticity(ne, young)
    perm, node_ptr, parent = w.grid_nested_dissection((ne + 1,) * 3, 27, dofs_per_point=3)
    N, _ = np.linalg.qr(w.rigid_modes(ne))
    n = K.shape[0]
    B = rng.standard_normal((n, 3))
    B -= N @ (N.T @ B)
    Xs = rng.standard_normal((n, 3))
    dE = young * rng.uniform(-1, 1, size=young.shape)
    opt = hy.hf_default_options(tau=1e-2, low_precision=32, gcr_block=0)
    ctx = hy.hf_analyse(K.indptr, K.indices, perm, node_ptr, parent, opt)
    dev = "cuda"
    Xs_t = torch.tensor(Xs, device=dev)
    Bt = torch.tensor(B, device=dev)

    def loss(vals):
        X = hy.solve(ctx, torch.tensor(vals, device=dev), Bt)
        return 0.5 * float(((X - Xs_t) ** 2).sum())

    v = torch.tensor(K.data, device=dev, requires_grad=True)
    X = hy.solve(ctx, v, Bt)
    (0.5 * ((X - Xs_t) ** 2).sum()).backward()
    gv = v.grad.cpu().numpy()
    h = 1e-5
    Kp, Km = w.q1_elasticity(ne, young + h * dE), w.q1_elasticity(ne, young - h * dE)
    assert np.array_equal(Kp.indices, K.indices) and np.array_equal(Km.indptr, K.indptr)
    dK = (Kp.data - Km.data) / (2 * h)
    fd = (loss(Kp.data) - loss(Km.data)) / (2 * h)
    print(f"  elasticity: moduli {gv @ dK:.10e} vs fd {fd:.10e}", flush=True)
    assert abs(gv @ dK - fd) <= 1e-5 * abs(fd)


@pytest.mark.parametrize("prec", [32, 64])
def test_autograd_stokes_viscosity(prec):
    """Enclosed MAC Stokes flow (zero pressure diagonal, saddle point): b is made
    at a reference viscosity field, the loss 0.5 ||x - x*||^2 is evaluated at
    another field.  The constant pressure stays the kernel for every viscosity,
    so the value gradient of hyfact.solve (through torch.autograd) chained to the
    per-cell viscosity (values = v0 + J mu) matches central differences of the
    GPU solve (h = 1e-6) and the oracle's gradient (dense adjoint)."""
    n = 8
    W = w.stokes_mac(n, seed=4, leaf_max=64, r=4)
    rng = np.random.default_rng(15)
    mu = W.meta["mu"] * np.exp(rng.uniform(-0.5, 0.5, size=W.meta["mu"].shape))
    J, v0 = w.mac_viscosity_jacobian(n)
    vals = v0 + J @ mu.reshape(-1, order="F")
    opt = hy.hf_default_options(tau=W.tau, low_precision=prec, gcr_block=0)
    ctx = hy.hf_analyse(W.indptr, W.indices, W.perm, W.node_ptr, W.parent, opt)
    dev = "cuda"
    Xs_t = torch.tensor(W.x_star, device=dev)
    Bt = torch.tensor(W.b, device=dev)

    def loss(m):
        v = v0 + J @ m.reshape(-1, order="F")
        X = hy.solve(ctx, torch.tensor(v, device=dev), Bt)
        return 0.5 * float(((X - Xs_t) ** 2).sum())

    v = torch.tensor(vals, device=dev, requires_grad=True)
    X = hy.solve(ctx, v, Bt)
    (0.5 * ((X - Xs_t) ** 2).sum()).backward()
    grad = J.T @ v.grad.cpu().numpy()
    d = mu * rng.uniform(-1, 1, size=mu.shape)
    h = 1e-6
    fd = (loss(mu + h * d) - loss(mu - h * d)) / (2 * h)
    an = float(grad @ d.reshape(-1, order="F"))
    # the oracle's gradient: dense adjoint on the same matrix
    import scipy.sparse as sp
    K = sp.csr_matrix((vals, W.indices, W.indptr), shape=(W.n, W.n))
    x = oracle.adjoint_solve(K, W.b, W.kernel)
    lam = oracle.adjoint_solve(K, x - W.x_star, W.kernel)
    gref = J.T @ oracle.value_gradient(W.indptr, W.indices, x, lam)
    rg = np.linalg.norm(grad - gref) / np.linalg.norm(gref)
    print(f"  prec {prec}: viscosity {an:.10e} vs fd {fd:.10e}; rel vs oracle gradient {rg:.2e}", flush=True)
    assert abs(an - fd) <= 1e-5 * abs(fd)
    assert rg <= 1e-9
