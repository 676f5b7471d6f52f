"""Write the full-size expected values used by the GPU tests (calls only the oracle).

For each single-GPU configuration (C2: 3D Neumann 64^3 with 200 inclusions, 16
right-hand sides; C3: floating Q1 elastic cube 24^3 elements, 32 right-hand
sides) the oracle runs Algorithms 1 and 2 in FP64 and records the hard-part size,
the hard part itself, the kernel dimension, a fixed sample of the minimum-norm
solution and its norm.  Usage: python tests/golden/make_golden.py c2 [c3 ...]
"""
import json
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


if __name__ == "__main__":
    for name in sys.argv[1:]:
        run(name)
