"""Postponing threshold of the 96-system batch (config c5), evaluated with the
oracle only.

Rule: the smallest tau of the threshold grid at which the single-precision step 1
of the oracle postpones at least one index of every system.  Each system is a
singular pure-Neumann Laplacian; with nothing postponed its whole, singular
matrix would be factorized, the FP32 rounding of the last pivot (up to 3e-4 of
the unit diagonal for these coefficient contrasts) standing in for the kernel's
zero.  Writes tests/golden/c5_tau.json: per threshold, every system's count of
postponed indices in FP32.  Run from the repository root:

    python tests/golden/make_c5_tau.py
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


def main():
    rng = np.random.default_rng(5)
    sides = rng.integers(16, 41, size=96)
    out = {"grid": list(w.C3_TAU_GRID), "sides": sides.tolist(), "M_fp32": {}}
    prepared = []
    for i, n in enumerate(sides):
        Wi = w.neumann3d(int(n), seed=5000 + i, leaf_max=512, r=1)
        q, K = oracle.scale(Wi.csr())
        Kp = oracle.permute(K, Wi.perm)
        prepared.append((Kp, Wi.node_ptr, Wi.parent, oracle.symbolic(Kp, Wi.node_ptr, Wi.parent)))
    for tau in w.C3_TAU_GRID:
        t0 = time.time()
        Ms = [int(len(oracle.factor_low(Kp, nptr, par, tau, dtype=np.float32, borders=bd).lambda2))
              for Kp, nptr, par, bd in prepared]
        out["M_fp32"][str(tau)] = Ms
        print(tau, "systems with nothing postponed:", sum(1 for m in Ms if m == 0), round(time.time() - t0, 1),
              flush=True)
        if min(Ms) >= 1:
            out["tau"] = tau
            break
    with open(os.path.join(ROOT, "tests", "golden", "c5_tau.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
