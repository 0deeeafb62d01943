"""Host logic of bench.py on the CPU: the HBM traffic model built from the
committed counters, and the one-GPU contract."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _points():
    with open(os.path.join(ROOT, "profiles", "k_smooth_fine_traffic.json")) as fh:
        J = json.load(fh)
    out = {}
    for p in J["points"]:
        out[p["slots"]] = 1024.0 * (p["fetch_kib"] * J["fetch_scale"] +
                                    p["write_kib"] * J["write_scale"])
    return J, out


def test_traffic_model_reproduces_its_measured_points():
    J, pts = _points()
    n = J["n"]
    if bench.traffic_per_launch(n, 1, n * 48.0) is None:
        pytest.skip("kernel sources changed since the counters were taken")
    for z, t in pts.items():
        launches = 100
        nbytes = launches * n * (32.0 * z + 16.0)   # the timer's accounting
        got = bench.traffic_per_launch(n, launches, nbytes)
        assert abs(got - t) <= 1e-9 * t, (z, got, t)


def test_traffic_model_refuses_another_grid():
    J, _ = _points()
    assert bench.traffic_per_launch(J["n"] + 1, 10, 1e9) is None
    assert bench.traffic_per_launch(J["n"], 0, 0.0) is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
