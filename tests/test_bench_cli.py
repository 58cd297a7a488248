"""bench.py's contract on the host: one GPU only, and the named workloads."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_workloads():
    import bench
    prob, params, desc = bench.workload("band4000")
    assert prob.n == prob.m == 4000 and params == {} and "bandwidth 20" in desc
    prob, params, desc = bench.workload("lattice400")
    assert prob.n == prob.m == 4000 and "p=400 q=10" in desc
    perm = params["user_perm"]
    assert np.array_equal(np.sort(perm), np.arange(4000))
