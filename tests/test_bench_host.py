"""Host logic of bench.py (CPU): the refusal of several GPUs and the roofline
arithmetic of the JSON line, on synthetic per-class counters."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "not supported" in p.stderr and "one GPU" in p.stderr


def _stats():
    # 2 steps: panel 10 ms (1 GB, 1 GFLOP), gram 1 ms (2 GB, 8 TFLOP -> FP64-bound), other empty
    return {"panel": {"ms": 10.0, "launches": 4, "bytes": 1e9, "flops": 1e9},
            "gram": {"ms": 1.0, "launches": 2, "bytes": 2e9, "flops": 8e12},
            "other": {"ms": 0.0, "launches": 0, "bytes": 0.0, "flops": 0.0}}


def test_path_roofline_sums_class_bounds():
    st = _stats()
    out = bench.path_roofline(st, 2, 32, 50.0)
    hbm = bench.PEAK["hbm_GBps"] * 1e9
    t_panel = max(1e9 / (bench.PEAK["fp32_TFLOPs"] * 1e12), 1e9 / hbm)
    t_gram = max(8e12 / (bench.PEAK["fp64_TFLOPs"] * 1e12), 2e9 / hbm)   # gram is an FP64 class
    assert out["t_roof_ms"] == pytest.approx((t_panel + t_gram) / 2 * 1e3)
    assert out["frac"] == pytest.approx(out["t_roof_ms"] / 50.0)
    assert set(out["per_class"]) == {"panel", "gram"}
    assert out["per_class"]["panel"]["hbm_frac"] == pytest.approx(1e9 / 0.010 / hbm, abs=1e-4)


def test_roofline_of_dominant_kernel():
    out = bench.roofline(_stats(), 2, 32)
    assert out["class"] == "panel" and out["bound"] == "hbm"
    assert out["achieved"] == pytest.approx(1e9 / 0.010 / 1e9)
    assert out["frac"] == pytest.approx(out["achieved"] / bench.PEAK["hbm_GBps"])
    assert out["avg_launch_ms"] == pytest.approx(2.5)
    assert out["bytes_per_launch"] == pytest.approx(2.5e8)
