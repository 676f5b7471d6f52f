"""Write the full-size expected values used by the GPU tests (calls only the oracle).

For each single-GPU configuration (C2: 3D Neumann 64^3 with 200 inclusions, 16
right-hand sides; C3: floating Q1 elastic cube 24^3 elements, 32 right-hand
sides) the oracle runs Algorithms 1 and 2 in FP64 and records the hard-part size,
the hard part itself, the kernel dimension, a fixed sample of the minimum-norm
solution and its norm.  With --nodes it writes the per-node record of step 1 in
FP32 and FP64 instead.  Usage: python tests/golden/make_golden.py [--nodes] c2 [c3 ...]
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2208_01907_amd import workloads as w  # noqa: E402

SAMPLE = 2048


def sample_rows(n, seed=99):
    return np.sort(np.random.default_rng(seed).choice(n, size=min(SAMPLE, n), replace=False))


def run(name):
    W = w.CONFIGS[name]()
    t0 = time.time()
    hf = oracle.hybrid_factorize(W.csr(), W.perm, W.node_ptr, W.parent, tau=W.tau, low=np.float64,
                                 gcr_block=0)
    X = oracle.hybrid_solve(hf, W.b)
    rows = sample_rows(W.n)
    out = {
        "config": name, "n": W.n, "tau": W.tau, "low": "fp64",
        "M": int(hf.M), "k": int(hf.k),
        "lambda2_original": sorted(int(x) for x in W.perm[hf.step1.lambda2]),
        "s22_pivot_mags": [float(x) for x in hf.ldl.mags],
        "gcr_iters": [int(x) for x in hf.gcr_iters],
        "sample_rows": rows.tolist(),
        "x_sample": X[rows].tolist(),
        "x_norm": float(np.linalg.norm(X)),
        "backward_error": oracle.backward_error(W.csr(), X, W.b),
        "seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle_fp64.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(name, "M", out["M"], "k", out["k"], "be", out["backward_error"], "s", out["seconds"])


def nodes(name):
    """Per-node step-1 record of the oracle in FP32 and in FP64 (Sec. 2.2 postponing).

    Writes {name}_oracle_nodes.json: accepted pivots per node in both precisions,
    the nodes whose FP32 decision is fixed independently of rounding
    (oracle.decided_nodes), and the last accepted pivots and the stopping
    candidate of the root in both precisions.
    """
    W = w.CONFIGS[name]()
    t0 = time.time()
    q, K = oracle.scale(W.csr())
    Kp = oracle.permute(K, W.perm)
    bd = oracle.symbolic(Kp, W.node_ptr, W.parent)
    f32 = oracle.factor_low(Kp, W.node_ptr, W.parent, W.tau, dtype=np.float32, borders=bd)
    f64 = oracle.factor_low(Kp, W.node_ptr, W.parent, W.tau, dtype=np.float64, borders=bd)
    dec, worst = oracle.decided_nodes(f32, f64, W.tau)
    root = len(W.parent) - 1

    def tail(f1):
        v, _ = oracle.tested_values(f1, root)
        n = int(f1.npiv[root])
        return {"npiv": n, "last_pivots": [float(x) for x in v[max(n - 12, 0):n]],
                "stop_candidate": None if math.isnan(float(f1.dstop[root])) else float(f1.dstop[root])}

    out = {
        "config": name, "n": W.n, "tau": W.tau, "n_nodes": len(W.parent),
        "npiv_fp32": [int(x) for x in f32.npiv], "npiv_fp64": [int(x) for x in f64.npiv],
        "M_fp32": int(f32.M), "M_fp64": int(f64.M),
        "decided": [bool(x) for x in dec],
        "tiegap_fp64": [float(x) if np.isfinite(x) else 1e300 for x in f64.tiegap],
        "worst_error_to_distance": [None if not np.isfinite(x) else float(x) for x in worst],
        "root": {"node": root, "fp32": tail(f32), "fp64": tail(f64)},
        "seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle_nodes.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(name, "M32", out["M_fp32"], "M64", out["M_fp64"], "undecided", int((~dec).sum()), "s", out["seconds"])


if __name__ == "__main__":
    # python tests/golden/make_golden.py c2 c3          -- FP64 solution goldens
    # python tests/golden/make_golden.py --nodes c2 c3  -- per-node step-1 records
    args = sys.argv[1:]
    if args and args[0] == "--nodes":
        for name in args[1:]:
            nodes(name)
    else:
        for name in args:
            run(name)
