"""Host-side checks of bench.py (no GPU): the one-GPU guard and the tt_round flop model."""
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
