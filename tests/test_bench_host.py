"""Host-side pieces of bench.py that run without a GPU: the oracle CPU
baseline on its own problem instance (any step count, independent of the
timed run's length), the byte counts behind the roofline, and the
single-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as W  # noqa: E402


def test_cpu_baseline_runs_more_steps_than_a_short_bench():
    """The driver's short run (--steps 20 --warmup 5) must not bound the
    oracle's step count: the baseline builds a problem of its own length."""
    r = bench.cpu_baseline(nsteps=30, n=512)
    assert r["kind"] == "oracle" and r["cores"] == 1
    assert r["value"] > 0 and r["seconds"] > 0
    h = r["host"]
    assert h["os_cpu_count"] >= 1 and h["cpus_available"] >= 1
    assert isinstance(h["cpu_model"], str)
    for d in h["blas_threads_during_timing"]:
        assert d["num_threads"] == 1


def test_unit_bytes_two_step_pair_c3():
    p = W.many_copies(nsteps=4)
    cells = 4096 * 4096
    mats = 4 * (128 + 128) ** 2          # one shared model
    assert bench.model_bytes(p) == mats
    assert bench.unit_bytes(p, 1, True) == 26 * cells + 2 * mats
    assert bench.unit_bytes(p, 1, False) == 26 * cells + mats
    assert bench.unit_bytes(p, 0, True) == 32 * cells + 2 * mats


def test_roofline_fields():
    p = W.many_copies(nsteps=4)
    r = bench.stencil_roofline(p, 100, 10.0, 1, True, 8, "vacuum")
    assert r["units"] == 50 and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["avg_unit_us"] - 200.0) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-3
    # the effective figure counts 24 B per cell-step, two steps per pair
    eff = r["effective"]
    assert eff["bytes_per_unit"] == 48 * 4096 * 4096 + 2 * bench.model_bytes(p)


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
