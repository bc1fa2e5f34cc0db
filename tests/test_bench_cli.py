"""bench.py command line on the CPU: more than one GPU is refused with a
message before anything touches a device."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_traffic_record_is_dropped_when_the_loop_source_changes(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "_loop_source_hash", lambda prec: "0" * 64)
    assert bench._traffic("rashba_s9_L24", "fp32") is None


def test_flop_counts_of_the_loop():
    """Survey count of the six-orbital loop per (q, k, channel): separable ky
    transform over 9 phases, halved by hermiticity, plus the block build
    (8 n_o^2 n_b (n_b + n_o^2)); matrix-core flops of the real-basis kernel:
    21 row tiles x 36 columns x 6 bands x 2, three BF16 products."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.credited_loop_flops_per_pair(6, 4) == 8 * 9 * 1296 // 2 + 8 * 36 * 6 * 42 == 119232
    assert bench.mfma_flops_per_pair(4) == 3 * 2 * 336 * 36 * 6
    assert bench.mfma_flops_per_pair(2) == 3 * 2 * 192 * 36 * 6
    model, n = bench._cpu_info()
    assert isinstance(model, str) and n >= 1
