"""Host-side checks of bench.py (no GPU): the one-GPU guard, the tt_round flop model
and the choice of the dominant kernel class."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_round_flop_model_two_cores_by_hand():
    # modes (3, 2), input ranks (1, 3, 1), output ranks (1, 2, 1):
    # left: absorb 2*1*1*3*3, QR(3x3) 2*3*9 - 18, absorb 2*3*3*2;
    # right: QR(3x2) 2*3*4 - 16/3, SVD 21*8, carry 2*3*2*2, absorb 2*1*3*3*2
    f = 18 + 36 + 36 + (24 - 16 / 3) + 168 + 24 + 36
    assert bench.round_model_flops([3, 2], [1, 3, 1], [1, 2, 1]) == pytest.approx(4 * f)


def test_round_flop_model_interior_core():
    # one more interior core of rank R adds the left sweep's 4R^3 + (4 - 2/3)R^3
    # (29.3 R^3 after the complex factor 4) and the right sweep's
    # (4 - 2/3)R^3 + 21R^3 + 4R^3 + 4R^3
    R = 64
    def fl(n):
        modes = [3] + [2] * (n - 1)
        rk = [1] + [R] * (n - 1) + [1]
        return bench.round_model_flops(modes, rk, rk)
    per_core = 4.0 * (4 + (4 - 2 / 3) + (4 - 2 / 3) + 21 + 4 + 4) * R ** 3
    assert fl(26) - fl(25) == pytest.approx(per_core, rel=1e-12)


def test_dominant_class_scales_the_svd_class_to_the_window():
    # class-timing iterations with 4 fallbacks' SVDs (120 SVD calls per
    # iteration, 300 ms) against a window without any: the GEMM dominates
    cls = {"gemm": {"ms": 75.0, "svd_calls": 120.0}, "qr": {"ms": 19.0, "svd_calls": 120.0},
           "svd": {"ms": 300.0, "svd_calls": 120.0}}
    assert bench.dominant_class(cls, 0.0) == ("gemm", 0.0)
    # a window with as many SVD calls as those iterations keeps the SVD's time
    assert bench.dominant_class(cls, 120.0) == ("svd", 300.0)
    # a third of them: 100 ms, still above the GEMM
    dom, ms = bench.dominant_class(cls, 40.0)
    assert dom == "svd" and ms == pytest.approx(100.0)
    # no SVDs in the class-timing iterations: the SVD class cannot dominate
    cls["svd"] = {"ms": 0.0, "svd_calls": 0.0}
    assert bench.dominant_class(cls, 3.0) == ("gemm", 0.0)
