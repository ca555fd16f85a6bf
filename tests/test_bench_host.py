"""bench.py plumbing that needs no GPU: every fixed-shape workload's seeded
input has the shape and dtype its entry declares, a measured-traffic lookup
for a workload without a counter summary gives None, and a multi-GPU request
is refused with a message."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

DTYPES = {"complex64": np.complex64, "float32 real": np.float32, "float64": np.float64}


@pytest.mark.parametrize("name", ["batch_c64", "short_c64", "real_f32", "plain_f64", "precision"])
def test_fixed_shape_inputs(name):
    w = bench.WORKLOADS[name]
    x = bench.make_inputs(name, w)
    assert x.shape == (w["batch"], w["N"])
    assert x.dtype == DTYPES[w["input"]]
    assert np.all(np.isfinite(x.view(np.float32 if x.dtype != np.float64 else np.float64)))


def test_inputs_are_seeded():
    w = bench.WORKLOADS["short_c64"]
    assert np.array_equal(bench.make_inputs("short_c64", w), bench.make_inputs("short_c64", w))


def test_traffic_lookup_without_summary():
    assert bench.measured_traffic("no_such_workload") is None


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
