"""Serving-path checks that need no GPU: the pool bookkeeping and the
admission policy (each built with g++ from its plain C++ header and run),
and the server API's argument checks, which return before any device call."""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pool_bookkeeping(tmp_path):
    exe = tmp_path / "pool_check"
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Werror",
                    os.path.join(ROOT, "tests", "host", "pool_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("OK")


def test_admission_policy(tmp_path):
    exe = tmp_path / "admit_check"
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Werror",
                    os.path.join(ROOT, "tests", "host", "admit_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("admission checks passed")


@pytest.mark.parametrize("field,value", [
    ("mode", 5), ("max_inflight", -1), ("max_inflight", 65), ("max_batch", -2), ("max_batch", 4097),
    ("max_queue", -1), ("flags", 4), ("flags", 0x200), ("batch_max_bins", -2), ("spin_us", -2),
    ("spin_us", 1000001),
])
def test_server_create_rejects_bad_config(field, value):
    import paper_2403_16665_amd as dd
    cfg = dd.dd_server_cfg(0, 0, 1 << 20, 0, 0, 0, 0, None)
    setattr(cfg, field, value)
    h = ctypes.c_void_p(99)
    assert dd._lib.dense_dft_server_create(ctypes.byref(cfg), ctypes.byref(h)) == 1
    assert not h.value


def test_server_null_arguments():
    import paper_2403_16665_amd as dd
    h = ctypes.c_void_p()
    assert dd._lib.dense_dft_server_create(None, ctypes.byref(h)) == 1
    cfg = dd.dd_server_cfg()
    assert dd._lib.dense_dft_server_create(ctypes.byref(cfg), None) == 1
    t = ctypes.c_uint64()
    r = dd.dd_result()
    d = dd.dd_desc(64, 2, 1.0, dd.DD_C64, 4096, 1 << 20)
    assert dd._lib.dense_dft_submit(None, ctypes.byref(d), ctypes.byref(t)) == 1
    assert dd._lib.dense_dft_submit_at(None, ctypes.byref(d), 0, ctypes.byref(t)) == 1
    assert dd._lib.dense_dft_poll(None, 1, ctypes.byref(r)) == 1
    assert dd._lib.dense_dft_wait(None, 1, 0, ctypes.byref(r)) == 1
    assert dd._lib.dense_dft_server_pause(None, 1) == 1
    assert dd._lib.dense_dft_server_stats(None, None) == 1
    assert dd._lib.dense_dft_server_destroy(None) == 1
    assert dd._lib.dense_dft_server_warm(None, 64, 2, 1.0, 1) == 1


def test_server_create_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2403_16665_amd as dd
    cfg = dd.dd_server_cfg(0, 0, 1 << 20, 0, 0, 0, 0, None)
    h = ctypes.c_void_p(5)
    assert dd._lib.dense_dft_server_create(ctypes.byref(cfg), ctypes.byref(h)) == 4  # DD_ERR_DEVICE
    assert not h.value


def test_clock_is_monotonic():
    import paper_2403_16665_amd as dd
    a = dd.dense_dft_clock_ns()
    b = dd.dense_dft_clock_ns()
    assert 0 < a <= b
