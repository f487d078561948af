"""Host-side logic of bench.py (no GPU): the one-GPU guard, the step-count
sizing and the rate helpers."""
import json
import os
import subprocess
import sys
import time
import types

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    msg = json.loads(res.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def _fake_torch():
    return types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))


def test_size_counts_keeps_given_counts_and_sizes_missing_ones():
    calls = []
    args = types.SimpleNamespace(steps=7, warmup=3)
    bench.size_counts(lambda: calls.append(1), args, _fake_torch())
    assert (args.steps, args.warmup) == (7, 3) and not calls  # nothing run
    args = types.SimpleNamespace(steps=None, warmup=None)
    bench.size_counts(lambda: calls.append(1), args, _fake_torch())
    # a step of a few microseconds: thousands of steps, capped at 5000
    assert 1000 <= args.steps <= 5000 and 500 <= args.warmup <= 5000 and len(calls) == 4
    # a 4 ms step: 40 ms of timed steps is 10, raised to the minimum of 50;
    # the given warmup stays
    args = types.SimpleNamespace(steps=None, warmup=2)
    bench.size_counts(lambda: time.sleep(0.004), args, _fake_torch())
    assert args.steps == 50 and args.warmup == 2


def test_hbm_rate_and_sized_run():
    r = bench.hbm_rate(6_291_456, 0.04, 14_993_408)
    assert abs(r["algorithmic_GBps"] - 157.2864) < 1e-6
    assert abs(r["measured_GBps"] - 374.8352) < 1e-6
    assert bench.hbm_rate(100, 1.0)["measured_GBps"] is None
    seen = []
    n, dt, out = bench._sized_run(lambda m: seen.append(m) or m, 1000, 10, 0.0)
    assert seen[0] == 10 and n == 10 and out == 10  # target 0 s: no growth
    cum = np.cumsum(np.arange(1, 101))
    n, _, _ = bench._sized_run(lambda m: m, 100, 5, 1e9, cum)
    assert n == 100  # a huge target is capped at the total


def test_roofline_names_the_kernel_of_the_tuned_tile():
    assert "gemm_direct_kernel" in bench.roofline_for("packed", 2, 1e9, 1.0, 12)["kernel"]
    wave = bench.roofline_for("packed", 4, 1e9, 1.0, 15)
    assert "gemm_wave_batched_kernel" in wave["kernel"]
    assert wave["achieved"] == pytest.approx(2.0 * 1e9 / 1e-3 / 1e12)  # 2 flop per mul-add
    assert "gemm_split_kernel" in bench.roofline_for("packed", 4, 1e9, 1.0, 14)["kernel"]
    assert "gemm_i8f_kernel" in bench.roofline_for("int8", 2, 1e9, 1.0, 5)["kernel"]
    rl = bench.roofline_for("packed", 2, 1024 ** 3, 0.03876, 12)
    assert abs(rl["frac"] - 2 * 1024 ** 3 / 0.03876e-3 / 78.6e12) < 1e-12
