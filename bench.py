"""Benchmark: mixed-precision hybrid factor+solve vs the same path in FP64, one MI355X.

Workload: 3D pure-Neumann 7-point FV Laplacian on a 64^3 grid (L = 262,144),
coefficient 1 with 200 random spherical inclusions (radius 2-6 cells) at 1e6,
geometric nested dissection (leaf 512), tau = 1e-2, 16 right-hand sides
b = K x*, x* ~ N(0,1) orthogonal to the constants (seeded, synthetic).

A step is one hf_factorize (Algorithm 1: FP32 step 1, FP64 block GCR for X12,
S22, FP64 rank-revealing LDL^T) plus one hf_solve (Algorithm 2) with the 16
right-hand sides; inputs are resident in HBM before the timed region.  The same
steps are then timed with the FP64 step 1 ("plain FP64 LDL^T" of the same
method).  Prints one JSON line.

--gpus N with N > 1 is not supported: this path runs on a single GPU.
"""
import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBps": 8000.0, "fp32_TFLOPs": 157.3, "fp64_TFLOPs": 78.6}
WORKLOADS = {
    "c1": "2D Neumann 5-point FV Laplacian 32x32 (L=1024), cell coefficients 10^U(-3,3), ND leaf 64, "
          "tau=1e-2, FP32 step 1 + FP64 block GCR, 1 RHS",
    "c2": "3D Neumann 7-point FV Laplacian 64^3 (L=262144), 200 inclusions at 1e6, ND leaf 512, tau=1e-2, "
          "FP32 step 1 + FP64 block GCR, 16 RHS",
    "c3": "floating Q1 elastic cube 24^3 elements (L=46875), E=10^U(0,6), nu=0.3, ND leaf 64 nodes, tau=0.2, "
          "FP32 step 1 + FP64 block GCR, 32 RHS",
    "c4": "enclosed MAC Stokes saddle point 32^3 cells (95232 face velocities + 32768 pressures, L=128000), "
          "viscosity 10^U(-2,2), staggered ND leaf 512, tau=1e-2, FP32 step 1 + FP64 block GCR, 32 RHS",
    "c5": "batch of 96 independent 3D Neumann 7-point FV Laplacians, sides n ~ U{16..40} (L=2326630 in all), "
          "cell coefficients 10^U(-3,3), one block-diagonal forest, ND leaf 512, tau=1e-2, FP32 step 1 + FP64 "
          "block GCR in 8-column blocks, 8 RHS per system",
}
CALIB_BYTES = 256 << 20
# measured HBM traffic of the dominant kernel (FETCH_SIZE / WRITE_SIZE passes),
# valid while the source file that holds the kernel is unchanged
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c2_inclusions64_fp32.json")
# classes that compute in FP64 whatever the factorization precision
FP64_CLASSES = {"spmm", "gram", "combine", "value_grad"}
KERNEL_NAME = {"panel": "k_panel", "permute_l11": "k_l11_gather + k_l11_back", "f11_update": "k_syrk (trailing F11)",
               "gather_border": "k_gather_border", "trsm": "k_trsm", "syrk": "k_syrk (contribution)",
               "extend_add": "k_extend_add", "fwd_diag": "k_fwd_diag", "fwd_update": "k_fwd_upd",
               "bwd_border": "k_bwd_border_part", "bwd_diag": "k_bwd_diag", "bwd_update": "k_bwd_upd",
               "spmm": "k_spmm_k11", "gram": "k_gram_partial", "combine": "k_combine",
               "fwd_front": "k_fwd_front", "bwd_front": "k_bwd_front"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="time the oracle on the whole workload whatever its size")
    ap.add_argument("--cpu-baseline-sample", action="store_true",
                    help="time the oracle on the subtree sample only")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="run only the oracle timing (no GPU) and print it as JSON")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the sweeps' launch shapes (hf_tune) before timing")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one plain device copy of 256 MiB (calibrates HBM byte counters)")
    return ap.parse_args()


def run_path(hy, W, vals, B, prec, steps, warmup, torch, tune=False):
    """Times `steps` factor+solve steps (after `warmup`), then repeats them with
    per-launch HIP events to collect the per-kernel times.  With tune, the
    sweeps' launch shapes are first autotuned (hf_tune) on the factors of one
    factorization, for the wider of the Schur-complement blocks and the
    right-hand sides; the choice and its cost are kept on the context."""
    opt = hy.hf_default_options(tau=W.tau, low_precision=prec, gcr_block=0)
    t0 = time.perf_counter()
    ctx = hy.hf_analyse(W.indptr, W.indices, W.perm, W.node_ptr, W.parent, opt)
    t_an = time.perf_counter() - t0
    if tune:
        hy.hf_factorize(ctx, vals)
        r = max(1, min(64, max(int(B.shape[1]), min(64, hy.hf_info(ctx)["M"]))))
        t0 = time.perf_counter()
        fm, wm, ms = hy.hf_tune(ctx, r)
        ctx.tuned = {"columns": r, "sweep_front_min": fm, "sweep_wide_min": wm, "ms_per_application": ms,
                     "tuning_s": time.perf_counter() - t0}
    for _ in range(warmup):
        hy.hf_factorize(ctx, vals)
        hy.hf_solve(ctx, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        hy.hf_factorize(ctx, vals)
        X = hy.hf_solve(ctx, B)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # the same steps with every launch bracketed by events
    hy.hf_timing_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        hy.hf_factorize(ctx, vals)
        X = hy.hf_solve(ctx, B)
    torch.cuda.synchronize()
    dt_ev = (time.perf_counter() - t0) / steps
    stats = hy.hf_timing_get(ctx)
    info = hy.hf_info(ctx)
    hy.hf_timing_enable(ctx, False)
    return ctx, X, dt, dt_ev, t_an, stats, info


# classes that hold several kernels are not priced as one kernel
MIXED_CLASSES = {"solve_gather", "other", "permute_l11"}


def rates(stats):
    """Algorithmic GB/s and TFLOP/s of every kernel class (event times)."""
    out = {}
    for k, v in stats.items():
        if v["ms"] > 0 and k not in MIXED_CLASSES:
            out[k] = {"GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1),
                      "TFLOP/s": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2)}
    return out


def measured_traffic(cls, prec):
    """HBM bytes per launch of the kernel class from the committed counter
    summary, or None when there is none for it or its source has changed."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("class") != cls or t.get("prec") != prec:
        return None
    src = os.path.join(ROOT, t["source"])
    try:
        with open(src, "rb") as fh:
            digest = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return None
    if digest != t.get("source_sha256"):
        return None
    return t["bytes_per_launch"]


def roofline(stats, steps, prec):
    """Roofline of the kernel with the largest summed time: algorithmic bytes
    and flops per launch (from the front sizes) over its average event time;
    the bound is whichever of HBM and the matrix/vector peak of its precision
    the algorithmic work reaches first."""
    name = max((k for k in stats if k not in MIXED_CLASSES), key=lambda k: stats[k]["ms"])
    s = stats[name]
    launches = max(s["launches"], 1)
    per_launch_ms = s["ms"] / launches
    prec_peak = PEAK["fp32_TFLOPs"] if (prec == 32 and name not in FP64_CLASSES) else PEAK["fp64_TFLOPs"]
    t_hbm = s["bytes"] / (PEAK["hbm_GBps"] * 1e9)
    t_fl = s["flops"] / (prec_peak * 1e12)
    sec = s["ms"] * 1e-3
    if t_fl > t_hbm:
        achieved = s["flops"] / sec / 1e12 if sec > 0 else 0.0
        out = {"bound": "mfma", "achieved": achieved, "peak": prec_peak, "unit": "TFLOP/s"}
    else:
        achieved = s["bytes"] / sec / 1e9 if sec > 0 else 0.0
        out = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_GBps"], "unit": "GB/s"}
    out["frac"] = out["achieved"] / out["peak"]
    out["traffic"] = measured_traffic(name, prec)
    out.update({"kernel": KERNEL_NAME.get(name, name), "class": name, "launches_per_step": s["launches"] / steps,
                "avg_launch_ms": per_launch_ms, "bytes_per_launch": s["bytes"] / launches,
                "flops_per_launch": s["flops"] / launches})
    return out


def path_roofline(stats, steps, prec, ms_per_step):
    """Roofline of the whole step: T_roof = sum over kernel classes of
    max(algorithmic flops / peak of the class's precision, algorithmic bytes /
    HBM peak), per step, against the measured step time; plus each class's
    fraction of the HBM and arithmetic peaks.  Classes that hold several kernels
    count with whatever algorithmic work they record."""
    t_roof = 0.0
    per = {}
    for k, v in stats.items():
        if v["ms"] <= 0:
            continue
        pk = PEAK["fp32_TFLOPs"] if (prec == 32 and k not in FP64_CLASSES) else PEAK["fp64_TFLOPs"]
        t_roof += max(v["flops"] / (pk * 1e12), v["bytes"] / (PEAK["hbm_GBps"] * 1e9)) / steps
        sec = v["ms"] * 1e-3
        per[k] = {"hbm_frac": round(v["bytes"] / sec / 1e9 / PEAK["hbm_GBps"], 4),
                  "peak_frac": round(v["flops"] / sec / 1e12 / pk, 4)}
    return {"t_roof_ms": t_roof * 1e3, "t_measured_ms": ms_per_step, "frac": t_roof * 1e3 / ms_per_step,
            "per_class": per}


def _subtree_sample(W, frac):
    """The nested-dissection subtree whose size is closest to frac * n, as a
    problem of its own (rows and columns of the permuted scaled matrix)."""
    import numpy as np
    import oracle
    q, K = oracle.scale(W.csr())
    Kp = oracle.permute(K, W.perm)
    n_nodes = len(W.parent)
    first = np.arange(n_nodes)
    for j in range(n_nodes):
        pj = W.parent[j]
        if pj >= 0:
            first[pj] = min(first[pj], first[j])
    sub_n = np.array([W.node_ptr[j + 1] - W.node_ptr[first[j]] for j in range(n_nodes)])
    j = int(np.argmin(np.abs(sub_n - frac * W.n)))
    lo, hi = first[j], j + 1
    s0, s1 = W.node_ptr[lo], W.node_ptr[hi]
    Ksub = Kp[s0:s1, s0:s1].tocsr()
    nptr = (W.node_ptr[lo:hi + 1] - s0).astype(np.int32)
    par = np.array([p - lo if (p >= 0 and p < hi) else -1 for p in W.parent[lo:hi]], dtype=np.int32)
    return j, Ksub, nptr, par


SAMPLE_SCRIPT = """
import sys, time, numpy as np, scipy.sparse as sp
sys.path.insert(0, {root!r})
import oracle
d = np.load({path!r})
K = sp.csr_matrix((d['data'], d['indices'], d['indptr']), shape=tuple(d['shape']))
bd = oracle.symbolic(K, d['nptr'], d['par'])
t0 = time.perf_counter()
oracle.factor_low(K, d['nptr'], d['par'], float(d['tau']), dtype=np.float32, borders=bd)
print(time.perf_counter() - t0)
"""


def _oracle_run(K, perm, node_ptr, parent, tau, B):
    """The oracle's FP32 factor+solve (Algorithm 1, then Algorithm 2 with the
    residual-correction pass), timed by phase."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    hf = oracle.hybrid_factorize(K, perm, node_ptr, parent, tau=tau, low=np.float32, gcr_block=0)
    t1 = time.perf_counter()
    oracle.hybrid_solve(hf, B)
    t2 = time.perf_counter()
    phases = {"step1_s": hf.seconds["step1"], "gcr_s": hf.seconds["gcr"], "s22_s": hf.seconds["s22"],
              "solve_s": t2 - t1}
    return t2 - t0, phases, int(hf.M), int(hf.k)


FULL_BASELINE_FILE = os.path.join(ROOT, "profiles", "oracle_c2_full.json")
# workloads up to this many unknowns get the oracle's whole factor+solve as the
# baseline (the 64^3 workload: about 40 s on the GPU machine's 16 host cores); larger
# ones the subtree sample
FULL_BASELINE_MAX_N = 300_000


def host_cpu():
    """Model name of the host CPU (from /proc/cpuinfo where there is one)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.machine()


def cpu_baseline(W, cfg, full=False):
    """The oracle (unchanged), timed on the host with OpenMP over all host cores.

    full=True: its whole factor+solve of the workload with the FP32 step 1,
    split by phase.  Otherwise (larger workloads): the same on the
    nested-dissection subtree holding about 1/8 of the unknowns, as a problem of
    its own (its principal submatrix, the workload's right-hand-side count),
    plus its step 1 on that subtree with one thread, with the committed record
    of a whole-workload run (profiles/oracle_c2_full.json) attached when it is
    for this workload."""
    import subprocess
    import tempfile
    import numpy as np
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    if full:
        total, phases, M, k = _oracle_run(W.csr(), W.perm, W.node_ptr, W.parent, W.tau, W.b)
        return {"value": total, "unit": "s", "cores": threads, "kind": "oracle",
                "sample": "the whole workload: oracle FP32 step 1 + FP64 block GCR + S22 + solve with one "
                          "correction pass, OpenMP over all host cores (the C step 1 and preconditioner; "
                          "NumPy/SciPy for the rest)",
                "phases": phases, "M": M, "kernel_dim": k}
    j, Ksub, nptr, par = _subtree_sample(W, 0.125)
    rng = np.random.default_rng(2208)
    Bs = Ksub @ rng.standard_normal((Ksub.shape[0], W.b.shape[1]))
    total, phases, M, k = _oracle_run(Ksub, np.arange(Ksub.shape[0], dtype=np.int32), nptr, par, W.tau, Bs)
    out = {"value": total, "unit": "s", "cores": threads, "kind": "oracle",
           "sample": f"oracle FP32 factor+solve (Algorithm 1, Algorithm 2 with one correction pass, "
                     f"{W.b.shape[1]} RHS) of the nested-dissection subtree at node {j}: its principal "
                     f"submatrix, {Ksub.shape[0]} of the workload's {W.n} unknowns, OpenMP over all host cores",
           "phases": phases, "M": M, "kernel_dim": k}
    try:
        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "sub.npz")
            np.savez(path, data=Ksub.data, indices=Ksub.indices, indptr=Ksub.indptr, shape=np.array(Ksub.shape),
                     nptr=nptr, par=par, tau=W.tau)
            env = dict(os.environ, OMP_NUM_THREADS="1")
            res = subprocess.run([sys.executable, "-c", SAMPLE_SCRIPT.format(root=ROOT, path=path)], env=env,
                                 capture_output=True, text=True, timeout=600, check=True)
            out["step1_s_1_thread"] = float(res.stdout.strip().splitlines()[-1])
    except (OSError, subprocess.SubprocessError, ValueError) as e:
        out["step1_1_thread_error"] = str(e)
    try:
        with open(FULL_BASELINE_FILE) as fh:
            rec = json.load(fh)
        if rec.get("workload") == cfg:
            out["full_workload_measured"] = rec
    except (OSError, ValueError):
        pass
    return out


def batch_gates(W, X):
    """Per-system gate numbers of a batch (block-diagonal forest): the largest
    backward error and the largest relative error against x* over its systems."""
    import numpy as np
    from paper_2208_01907_amd.metrics import backward_error
    K = W.csr()
    offs = W.meta["offsets"]
    be, rel = [], []
    for i in range(len(offs) - 1):
        a, b = offs[i], offs[i + 1]
        be.append(backward_error(K[a:b, a:b], X[a:b], W.b[a:b]))
        rel.append(float(np.linalg.norm(X[a:b] - W.x_star[a:b]) / np.linalg.norm(W.x_star[a:b])))
    return {"systems": len(offs) - 1, "backward_error_max": max(be), "gate_1e-14_every_system": bool(max(be) <= 1e-14),
            "rel_err_vs_xstar_max": max(rel)}


def golden_rel(cfg, X):
    """Relative difference between X and the oracle's FP64 minimum-norm solution
    stored for this workload (tests/golden, written by the oracle), over the
    stored sample of rows; None when no stored solution exists."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{cfg}_oracle_fp64.json")
    try:
        with open(path) as fh:
            g = json.load(fh)
    except (OSError, ValueError):
        return None
    rows = np.array(g["sample_rows"])
    xs = np.array(g["x_sample"])
    return {"value": float(np.linalg.norm(X[rows] - xs) / np.linalg.norm(xs)), "rows": int(len(rows)),
            "reference": f"oracle FP64 solution (tests/golden/{cfg}_oracle_fp64.json)"}


def adjoint_timing(hy, ctx, X, W, steps, torch):
    """hf_adjoint on the factors of the last step (not part of the metric): one
    more Algorithm 2 solve for a seeded loss gradient G = dl/dX, then the value
    gradient on the pattern, whose kernel is priced against the HBM peak."""
    import numpy as np
    G = torch.tensor(np.random.default_rng(2208).standard_normal(W.b.shape), device=X.device)
    hy.hf_adjoint(ctx, X, G)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        hy.hf_adjoint(ctx, X, G)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    hy.hf_timing_enable(ctx, True)
    for _ in range(steps):
        hy.hf_adjoint(ctx, X, G)
    torch.cuda.synchronize()
    st = hy.hf_timing_get(ctx)["value_grad"]
    hy.hf_timing_enable(ctx, False)
    ms = st["ms"] / max(1, st["launches"])
    gbs = st["bytes"] / max(1, st["launches"]) / (ms * 1e-3) / 1e9 if ms > 0 else None
    return {"ms_per_call": dt * 1e3, "rhs": int(W.b.shape[1]),
            "value_grad": {"kernel": "k_value_grad", "avg_launch_ms": ms,
                           "bytes_per_launch": st["bytes"] / max(1, st["launches"]),
                           "achieved_GBps": gbs, "peak_GBps": PEAK["hbm_GBps"],
                           "frac": gbs / PEAK["hbm_GBps"] if gbs else None}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this hybrid-factorization path runs on one GPU "
              "(sharding over GPUs by nested-dissection subtrees is not built).",
              file=sys.stderr)
        sys.exit(2)
    if args.cpu_baseline_only:  # host only: the oracle's timing, no GPU
        from paper_2208_01907_amd import workloads as w
        W = w.CONFIGS[args.config]()
        rec = cpu_baseline(W, args.config, full=args.cpu_baseline_full or (W.n <= FULL_BASELINE_MAX_N and
                                                                          not args.cpu_baseline_sample))
        rec.update({"workload": args.config, "host": host_cpu(),
                    "command": " ".join(["python", "bench.py"] + sys.argv[1:])})
        print(json.dumps(rec))
        return
    import numpy as np
    import torch
    from paper_2208_01907_amd import hyfact as hy
    from paper_2208_01907_amd import workloads as w

    W = w.CONFIGS[args.config]()
    dev = torch.device("cuda:0")
    if args.calib_copy:
        src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    vals = torch.tensor(W.values, device=dev)
    B = torch.tensor(W.b, device=dev)
    torch.cuda.synchronize()
    ctx, X, dt, dt_ev, t_an, stats, info = run_path(hy, W, vals, B, hy.HF_PREC_FP32, args.steps, args.warmup,
                                                     torch, tune=args.tune)
    Xh = X.cpu().numpy()
    from paper_2208_01907_amd.metrics import backward_error
    be = backward_error(W.csr(), Xh, W.b)
    rel_xstar = float(np.linalg.norm(Xh - W.x_star) / np.linalg.norm(W.x_star))
    rel_oracle = golden_rel(args.config, Xh)
    result = {
        "metric": "factor+solve s at backward err <=1e-14, mixed vs FP64 LDL^T; % HBM/MFMA peak",
        "value": dt, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "n": W.n, "nnz": W.nnz, "rhs": int(W.b.shape[1])},
        "M": info["M"], "kernel_dim": info["kernel_dim"], "gcr_iters_max": info["gcr_iters_max"],
        "solve_gcr_iters": info["solve_gcr_iters"], "backward_error": be, "gate_1e-14": bool(be <= 1e-14),
        "rel_err_vs_xstar": rel_xstar, "rel_vs_oracle": rel_oracle, "gate_rel_1e-10": (
            None if rel_oracle is None else bool(rel_oracle["value"] <= 1e-10)), "analyse_s": t_an, "ms_per_step_with_events": dt_ev * 1e3,
        "phase_ms": {k: info[k] for k in ("t_step1_ms", "t_gcr_ms", "t_s22_ms", "t_solve_ms")},
        "kernel_ms_per_step": {k: v["ms"] / args.steps for k, v in stats.items()},
        "kernel_rates": rates(stats),
        "roofline": roofline(stats, args.steps, 32),
        "path_roofline": path_roofline(stats, args.steps, 32, dt * 1e3),
    }
    if getattr(ctx, "tuned", None):
        result["tuned"] = ctx.tuned
    if "offsets" in W.meta:  # a batch: the gate holds for every system on its own
        result["batch"] = batch_gates(W, Xh)
    result["adjoint"] = adjoint_timing(hy, ctx, X, W, args.steps, torch)
    del ctx
    if not args.no_fp64:
        ctx64, X64, dt64, dt64_ev, _, stats64, info64 = run_path(hy, W, vals, B, hy.HF_PREC_FP64, args.steps,
                                                                 args.warmup, torch)
        X64h = X64.cpu().numpy()
        be64 = backward_error(W.csr(), X64h, W.b)
        result["fp64"] = {"what": "the same pipeline (Algorithm 1, Algorithm 2 with the correction pass) with an "
                                  "FP64 step 1: the supernodal LDL^T in FP64, after which block GCR needs one "
                                  "iteration",
                          "s_per_step": dt64, "s_per_step_with_events": dt64_ev, "M": info64["M"],
                          "kernel_dim": info64["kernel_dim"],
                          "backward_error": be64, "rel_vs_oracle": golden_rel(args.config, X64h),
                          "kernel_ms_per_step": {k: v["ms"] / args.steps for k, v in stats64.items()},
                          "kernel_rates": rates(stats64),
                          "roofline": roofline(stats64, args.steps, 64),
                          "path_roofline": path_roofline(stats64, args.steps, 64, dt64 * 1e3)}
        result["speedup_vs_fp64"] = dt64 / dt
        del ctx64
    if not args.no_fp16:
        result["fp16_updates"] = {}
        for key, prec, what in (
                ("pair", hy.HF_PREC_FP16_PAIR, "FP32 fronts; trailing and contribution updates on the FP16 matrix "
                 "cores with operands as FP16 pairs (three products), per-tile 2^k scaling, FP32 accumulation"),
                ("single", hy.HF_PREC_FP16, "as pair, operands rounded to single FP16 numbers (one product)")):
            try:
                ctx16, X16, dt16, dt16_ev, _, stats16, info16 = run_path(hy, W, vals, B, prec, args.steps,
                                                                         args.warmup, torch)
            except hy.HFError as e:
                result["fp16_updates"][key] = {"what": what, "error": str(e)}
                continue
            X16h = X16.cpu().numpy()
            runs16, nfac16 = hy.hf_gcr_history(ctx16)
            result["fp16_updates"][key] = {
                "what": what, "s_per_step": dt16, "speedup_vs_fp32_updates": dt / dt16, "M": info16["M"],
                "kernel_dim": info16["kernel_dim"], "gcr_iters_max": info16["gcr_iters_max"],
                "solve_gcr_iters": info16["solve_gcr_iters"],
                "gcr_histories": [[float(x) for x in r] for r in runs16],
                "backward_error": backward_error(W.csr(), X16h, W.b),
                "rel_vs_oracle": golden_rel(args.config, X16h),
                "kernel_ms_per_step": {k: v["ms"] / args.steps for k, v in stats16.items()},
                "kernel_rates": rates(stats16)}
            del ctx16
    if not args.no_cpu_baseline:
        full = args.cpu_baseline_full or (W.n <= FULL_BASELINE_MAX_N and not args.cpu_baseline_sample)
        result["cpu_baseline"] = cpu_baseline(W, args.config, full=full)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
