"""The library driven from PyTorch: device tensors as inputs and outputs and
torch's current HIP stream as the context stream (in a subprocess that
imports torch first, so one HIP runtime serves both)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
HELPER = os.path.join(os.path.dirname(__file__), "helpers", "torch_solve.py")


def test_solve_from_torch_tensors_on_torch_stream():
    r = subprocess.run([sys.executable, HELPER], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    print(res)
    assert res["iters"] == res["iters_host"]
    assert res["u_diff"] <= 1e-14 and res["spmv_diff"] <= 1e-14
    assert abs(res["norm_dev"] / res["norm_host"] - 1) <= 1e-14
