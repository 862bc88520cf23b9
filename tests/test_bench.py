"""Host logic of bench.py (no GPU): the one-GPU guard, the oracle CPU-baseline
samplers on small grids, and the lookup of measured HBM traffic (keyed by the
kernel sources' hash and the coarse restart)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2308_06152_amd import inputs  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _check_line(c):
    assert c["kind"] == "oracle" and c["unit"] == "solves/s"
    assert c["value"] > 0 and c["value_1thread"] > 0 and c["cores"] >= 1
    assert isinstance(c["sample"], str) and c["sample"]


def test_cpu_baseline_whole_solves_small_grid():
    w = inputs.scaled_plain(33, 5.0)
    c = bench.cpu_baseline_full(w, 0, w.coarse_restart, reps=1)
    _check_line(c)
    assert "whole oracle solves" in c["sample"]


def test_cpu_baseline_sample_extrapolates_with_the_run_counts():
    w = inputs.scaled_plain(65, 10.0)
    c1 = bench.cpu_baseline(w, {"outer_iters": 2, "inner_iters_total": 20}, 0, 5)
    c2 = bench.cpu_baseline(w, {"outer_iters": 2, "inner_iters_total": 2000}, 0, 5)
    _check_line(c1)
    _check_line(c2)
    assert "coarse restart 5" in c1["sample"]
    # a hundred times the inner iterations: a much longer estimated solve
    assert c2["est_seconds_per_solve"] > 5 * c1["est_seconds_per_solve"]


def test_measured_traffic_lookup(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    sha = bench.kernels_hash()
    f.write_text(json.dumps({
        "mupdate@wl": {"kernels_sha": sha, "bytes_per_launch": 5.0, "coarse_restart": 10},
        "mdot@wl": {"kernels_sha": "0" * 16, "bytes_per_launch": 7.0},
    }))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("mupdate", "wl", 10) == 5.0
    assert bench.measured_traffic("mupdate", "wl", 15) is None   # another restart
    assert bench.measured_traffic("mdot", "wl", 10) is None      # other kernel sources
    assert bench.measured_traffic("apply5", "wl", 10) is None    # not measured
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("mupdate", "wl", 10) is None
