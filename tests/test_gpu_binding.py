"""The binding in a fresh process: a host-only library call made before
anything imports torch still leaves one HIP runtime in the process, so a
context created afterwards sees the device and solves."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
import numpy as np
from paper_1603_09311_amd import sdd, workloads as W
assert "torch" not in sys.modules
e = np.array([1.0 + 0.5j, 0.8 + 0.2j])
rho, phi = sdd.mt_te_response(e * 1.01, e, e * 0.99, 0.01, 1000.0, 10.0)
print("host call done", rho, flush=True)
ctx = sdd.Context(0, workspace_bytes=1 << 30)
p = W.unit_square(n_nodes=4)
r = ctx.solve(p)
assert r["paths_done"].sum() == p.path_count.sum(), r["paths_done"]
ctx.close()
print("solved", r["mean"], flush=True)
"""


def test_host_call_before_torch_then_solve():
    out = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True, text=True, timeout=100)
    print(out.stdout, out.stderr[-2000:], flush=True)
    assert out.returncode == 0
    assert "solved" in out.stdout
