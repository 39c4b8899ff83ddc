"""The benchmark's contract on the host (no GPU): the method's algorithmic
bytes per cell of each workload, the refusal of more than one GPU, and that
the committed counter summaries were taken on the current kernel sources (a
change to the kernels must come with new counters)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("setup,expected", [
    (dict(dim=3, precision="fp32", ns=4), 244.0),   # one-step sphere bed
    (dict(dim=3, precision="fp32", ns=9), 284.0),   # nine-species beds
    (dict(dim=2, precision="fp64", ns=0), 248.0),   # cylinder channel
])
def test_method_bytes_per_cell(setup, expected):
    assert bench.method_bytes_per_cell(setup) == expected


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("name", ["sphere_bed", "superquadric_bed"])
def test_counter_summaries_match_the_kernel_sources(name):
    d = json.load(open(os.path.join(ROOT, "profiles", f"traffic_{name}.json")))
    assert d["kernel_hash"] == bench.kernel_hash()
    assert os.path.exists(os.path.join(ROOT, "profiles", d["summary"]))
    # HBM bytes per launch within a few tens of percent of the algorithmic ones
    assert 1.0 <= d["bytes_per_launch"] / d["bytes_per_launch_alg"] < 1.5
    alu = bench.alu_from_profiles(name, d["bytes_per_launch_alg"], 1.0)
    assert alu is not None and alu["bound"] == "alu" and 0 < alu["frac"]
    assert bench.traffic_from_profiles(name, d["bytes_per_launch_alg"]) == d["bytes_per_launch"]
    assert bench.traffic_from_profiles(name, d["bytes_per_launch_alg"] + 1) is None
