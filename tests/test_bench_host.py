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


def test_streaming_legs_cycle_buffer_sets_past_the_cache(monkeypatch):
    # enough sets that the timed steps touch over four times the 256 MiB
    # Infinity Cache; --rotate overrides; every set is written once before
    # the timed steps, which then take the sets in turn
    args = types.SimpleNamespace(rotate=0, steps=5, warmup=2)
    assert len(bench.rotating_sets(lambda i: i, 184_549_376, args)) == 6
    assert len(bench.rotating_sets(lambda i: i, 2 << 30, args)) == 2  # at least two
    assert len(bench.rotating_sets(lambda i: i, 65536 * 11, args)) == 64  # at most 64
    args.rotate = 3
    sets = bench.rotating_sets(lambda i: i, 184_549_376, args)
    assert sets == [0, 1, 2]
    seen = []

    def fake_time_steps(fn, steps, warmup, torch):
        for _ in range(warmup + steps):
            fn()
        return 1.0

    monkeypatch.setattr(bench, "time_steps", fake_time_steps)
    ms, one = bench.time_rotating(lambda x: seen.append(x), [(i,) for i in sets], args,
                                  _fake_torch())
    assert (ms, one) == (1.0, 1.0)
    cycled = [0, 1, 2] + [i % 3 for i in range(7)]  # fill, then warmup + steps in turn
    assert seen[:10] == cycled and seen[10:] == [0] * 7  # then the first set alone


def test_transform_inputs_are_exact_and_in_range():
    from paper_0710_0510_amd import workloads as W
    w = W.Workload("t", "transforms", 5, 3, (3, 3, 0), seed=9, n=5000, q=64)
    c, r = W.transform_inputs(w)
    assert c.shape == (5000, 3) and c.dtype == np.uint8 and int(c.max()) < 5
    assert r.dtype == np.float64 and (r == np.floor(r)).all()
    assert float(r.min()) >= 0 and float(r.max()) < 64 ** 5
    c2, r2 = W.transform_inputs(w)
    assert np.array_equal(c, c2) and np.array_equal(r, r2)  # seeded
    assert W.WORKLOADS["transforms-gf5^3-2^24"].q ** 5 <= 2 ** 53
