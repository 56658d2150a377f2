"""Host-side pieces of bench.py that need no GPU: the oracle's time to the
certified gap on one core (the small configuration's CPU baseline), the
per-mode workload defaults, and the algorithmic byte counts."""

import os
import subprocess
import sys

import numpy as np
import pytest

import bench
import oracle
from workloads import make_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("tau", [1, 8])
def test_oracle_time_to_gap_certifies(tau):
    inst = make_config("small_2000x1000", dtype="f64")
    r = bench.oracle_time_to_gap(inst.A, inst.b, inst.lam, tau, 1e-6, 60.0)
    assert r["reached"] and r["rel_gap"] <= 1e-6 and r["cores"] == 1
    assert 1 <= r["gap_evaluations"] <= r["epochs"]
    # the same number of epochs from x = 0, recomputed without the schedule
    ref = oracle.Solver(inst.A, inst.b, inst.lam, tau=tau, seed=0)
    ref.step(r["epochs"] * ref.steps_per_epoch())
    gap, F, D = ref.gap()
    assert gap / abs(D) == pytest.approx(r["rel_gap"], rel=1e-9, abs=1e-15)


def test_algorithmic_bytes_per_update():
    """268 B gather / 160 B scatter per update for d = 20 float32 values; 228 /
    160 for bf16 (the per-update figures the roofline uses)."""
    g, sc = bench.algorithmic_bytes(20, 4)
    assert (g, sc) == (268, 160)
    g, sc = bench.algorithmic_bytes(20, 2)
    assert (g, sc) == (228, 160)


@pytest.mark.parametrize("mode", ["dtypes", "samplings", "async"])
def test_host_built_modes_refuse_the_device_generated_instance(mode):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--mode", mode, "--config", "lasso_2e8x5e8"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "generated on the device only" in r.stderr


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
