"""bench.py's host-side contract (no GPU): the one-GPU rule, the workload
table, and the oracle leg it times on the host."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_several_gpus_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_workloads_and_description():
    assert set(bench.WORKLOADS) == {"nldiff512-gauss3", "nldiff1024-gauss5", "vsf1024-radau3"}
    problem, n, family, s, dt, steps, nu = bench.WORKLOADS["nldiff512-gauss3"]
    assert (problem, n, family, s, dt, steps) == ("nldiff", 512, "gauss", 3, 5e-3, 50)
    d = bench.describe(*bench.WORKLOADS["vsf1024-radau3"])
    assert "1024x1024" in d and "Radau IIA s=3" in d and "20 steps" in d


@pytest.mark.parametrize("name,n", [("nldiff512-gauss3", 12), ("vsf1024-radau3", 8)])
def test_cpu_baseline_leg(name, n):
    """The oracle leg on a tiny sample: one full-Newton step, one thread."""
    out = bench.cpu_baseline(bench.WORKLOADS[name], n)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "DOF*stages/s"
    assert out["value"] > 0 and f"{n}x{n}" in out["sample"]
