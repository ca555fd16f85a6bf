"""C ABI checks that need no GPU: the library loads, exports every function
include/dense_dft.h declares, and rejects bad arguments before any device call."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dense_dft.h")
LIB = os.path.join(ROOT, "paper_2403_16665_amd", "libdensedft.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dense_dft_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (dense_dft_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    assert len(declared_functions()) >= 8


def test_binding_loads_and_names_match():
    import paper_2403_16665_amd as dd
    for f in declared_functions():
        assert hasattr(dd._lib, f)
        assert hasattr(dd, f), f"binding lacks {f}"
    assert dd.dense_dft_version() >= 100
    assert dd.dense_dft_status_string(0) == "ok"
    assert "unsupported" in dd.dense_dft_status_string(2)


@pytest.mark.parametrize("N,alpha,T,batch,dtype,flags,want", [
    (0, 2, 1.0, 1, 1, 0, 1),                 # N < 1
    (64, 2, 0.0, 1, 1, 0, 1),                # T <= 0
    (64, 2, float("inf"), 1, 1, 0, 1),       # T not finite
    (64, 2, float("nan"), 1, 1, 0, 1),
    (64, 2, 1.0, 0, 1, 0, 1),                # batch < 1
    (64, 2, 1.0, 1, 7, 0, 1),                # bad dtype
    (64, 2, 1.0, 1, 1, 8, 1),                # unknown flag
    (64, 0, 1.0, 1, 1, 0, 2),                # alpha < 1 (alpha < 1 is a one-way transform; unsupported)
    (64, -3, 1.0, 1, 1, 0, 2),
    (7, 2, 1.0, 1, 1, 0, 2),                 # prime factor > 5
    (15 * 4096, 2, 1.0, 1, 1, 0, 2),         # 3 and 5 in one length: not a built length
    (1 << 25, 2, 1.0, 1, 1, 0, 2),           # beyond 4096 x 4096
    (1 << 24, 2, 1.0, 1, 2, 0, 2),           # double: 4096 x 4096 needs a column of 4096 in LDS
    (1 << 24, 2, 1.0, 1, 3, 0, 2),
    (1 << 20, 4096, 1.0, 1, 1, 0, 2),        # alpha*N > 2^31
    (64, 2, 1e300, 1, 1, 0, 2),              # T/N beyond float: every bin would be infinite
    (64, 2, 1e300, 1, 0, 0, 2),
    (64, 2, 1e-40, 1, 1, 0, 2),              # T/N below float's normal range
    (64, 2, 1e-310, 1, 3, 0, 2),             # T/N below double's normal range
])
def test_plan_rejects_bad_arguments(N, alpha, T, batch, dtype, flags, want):
    import ctypes
    import paper_2403_16665_amd as dd
    h = ctypes.c_void_p(12345)
    rc = dd._lib.dense_dft_plan(ctypes.byref(h), N, alpha, T, batch, dtype, flags)
    assert rc == want
    assert not h.value  # out-param cleared on failure


@pytest.mark.parametrize("dtype,n1_4096", [(0, True), (1, True), (2, False), (3, False)])
def test_schedules_fit_workgroup_lds(dtype, n1_4096):
    """A pass-1 column of 4096 fits a workgroup's LDS in single precision
    only: in double the planner neither offers nor accepts that schedule."""
    import ctypes
    import paper_2403_16665_amd as dd
    two = [sc for sc in dd.dense_dft_sched_candidates(8192, 2, 3, dtype) if sc.passes == 2]
    assert two
    assert any(sc.N1 == 4096 for sc in two) == n1_4096
    if not n1_4096:
        h = ctypes.c_void_p(12345)
        sc = dd.make_sched(2, N1=4096, N2=2)
        rc = dd._lib.dense_dft_plan_sched(ctypes.byref(h), 8192, 2, 1.0, 3, dtype, dd.DD_TWIDDLE_FP64,
                                          ctypes.byref(sc))
        assert rc == 2 and not h.value


def test_chunk_candidates():
    """Two-pass candidates with every j per block also come with 1.5x and 2x
    the default chunk (32 signals of 4 MiB scratch here), within the batch."""
    import paper_2403_16665_amd as dd
    chunks = {sc.chunk for sc in dd.dense_dft_sched_candidates(65536, 8, 256, 1)
              if sc.passes == 2 and sc.N1 == 256 and sc.jgroup == 8}
    assert chunks == {32, 48, 64}
    chunks = {sc.chunk for sc in dd.dense_dft_sched_candidates(65536, 8, 40, 1)
              if sc.passes == 2 and sc.N1 == 256 and sc.jgroup == 8}
    assert chunks == {32}


def test_schedules_fit_one_dispatch():
    """A launch's grid is a 32-bit count of work-items, so a schedule whose
    pass-1 grid would exceed 2^31 of them is neither offered nor accepted:
    at N = 4, alpha = 2^28 one j per block would take 2^28 blocks per
    signal, and a requested chunk of 2^31 signals of N = 8 as many blocks."""
    import ctypes
    import paper_2403_16665_amd as dd
    two = [sc for sc in dd.dense_dft_sched_candidates(4, 1 << 28, 1, 1) if sc.passes == 2]
    # blocks of at least one wave: 2^28 / jgroup blocks of 64 work-items fit only for jgroup >= 8
    assert two and all(sc.jgroup >= 8 for sc in two), sorted({sc.jgroup for sc in two})
    assert any(sc.jgroup == 1 for sc in dd.dense_dft_sched_candidates(4, 1 << 12, 1, 1) if sc.passes == 2)
    for dtype in (0, 1, 2, 3):
        h = ctypes.c_void_p(12345)
        sc = dd.make_sched(2, N1=2, N2=4, chunk=1 << 31)
        rc = dd._lib.dense_dft_plan_sched(ctypes.byref(h), 8, 1, 1.0, 1 << 31, dtype, dd.DD_TWIDDLE_FP64,
                                          ctypes.byref(sc))
        assert rc == 2 and not h.value


def test_null_handles_rejected():
    import ctypes
    import paper_2403_16665_amd as dd
    assert dd._lib.dense_dft_plan(None, 64, 2, 1.0, 1, 1, 0) == 1
    assert dd._lib.dense_dft_exec(None, None, None, None, None) == 1
    assert dd._lib.dense_dft_destroy(None) == 1
    n = ctypes.c_size_t()
    assert dd._lib.dense_dft_workspace_size(None, ctypes.byref(n)) == 1
    assert dd._lib.dense_dft_plan_info(None, None, None, None) == 1
    assert dd._lib.dense_dft_profile_begin(None, 4) == 1


def test_batch_plan_rejects_bad_descriptors():
    import ctypes
    import paper_2403_16665_amd as dd
    h = ctypes.c_void_p(7)
    ok = dd.dd_desc(1024, 4, 1.0, dd.DD_C64, 4096, 1 << 20)
    arr = (dd.dd_desc * 1)(ok)
    assert dd._lib.dense_dft_batch_plan(ctypes.byref(h), arr, 0, 0) == 1          # count < 1
    assert not h.value
    assert dd._lib.dense_dft_batch_plan(None, arr, 1, 0) == 1                     # null out
    assert dd._lib.dense_dft_batch_plan(ctypes.byref(h), None, 1, 0) == 1        # null descs
    for bad in [dd.dd_desc(0, 4, 1.0, dd.DD_C64, 4096, 1 << 20),                  # N < 1
                dd.dd_desc(1024, 4, -1.0, dd.DD_C64, 4096, 1 << 20),              # T <= 0
                dd.dd_desc(1024, 4, 1.0, 9, 4096, 1 << 20),                       # dtype
                dd.dd_desc(1024, 4, 1.0, dd.DD_C64, None, 1 << 20),               # null x
                dd.dd_desc(1024, 4, 1.0, dd.DD_C64, 4100, 1 << 20),               # misaligned x
                dd.dd_desc(1024, 4, 1.0, dd.DD_C64, 4096, 4096 + 8)]:             # x and X overlap
        assert dd._lib.dense_dft_batch_plan(ctypes.byref(h), (dd.dd_desc * 1)(bad), 1, 0) == 1
    for bad in [dd.dd_desc(1024, 0, 1.0, dd.DD_C64, 4096, 1 << 20),               # alpha < 1
                dd.dd_desc(7 * 64, 2, 1.0, dd.DD_C64, 4096, 1 << 20),             # prime factor 7
                dd.dd_desc(1024, 4, 1e300, dd.DD_C64, 4096, 1 << 20)]:            # T/N beyond float
        assert dd._lib.dense_dft_batch_plan(ctypes.byref(h), (dd.dd_desc * 1)(bad), 1, 0) == 2
    assert dd._lib.dense_dft_batch_exec(None, None) == 1
    assert dd._lib.dense_dft_batch_destroy(None) == 1


@pytest.mark.parametrize("N,p,want", [(12, 0, 2), (12, 5, 2), (61440 * 4, 4, 2), (0, 1, 1)])
def test_decimated_plan_rejects(N, p, want):
    import ctypes
    import paper_2403_16665_amd as dd
    h = ctypes.c_void_p(3)
    assert dd._lib.dense_dft_plan_decimated(ctypes.byref(h), N, p, 1.0, 1, dd.DD_C64, 0) == want
    assert not h.value


def test_binding_checks_tensors_before_the_library():
    """The binding refuses host tensors, wrong dtypes and short buffers with
    DD_ERR_INVALID before any library call (the plan here has no handle, so
    reaching the library would fail differently)."""
    import torch
    import paper_2403_16665_amd as dd
    fake = dd.Plan(None, 1024, 4, 1.0, 3, dd.DD_C64, 0)
    x = torch.zeros(3, 1024, dtype=torch.complex64)
    X = torch.zeros(3, 4096, dtype=torch.complex64)
    for call in (lambda: dd.dense_dft_exec(fake, x, X),
                 lambda: fake.exec(x, out=X),
                 lambda: dd.dense_dft_exec_inverse(fake, X, x),
                 lambda: dd._one_desc((1024, 4, 1.0, dd.DD_C64, x[0], X[0])),
                 lambda: dd._desc_array([(1024, 4, 1.0, dd.DD_C64, x[0], X[0])])):
        with pytest.raises(dd.DenseDFTError) as e:
            call()
        assert e.value.status == 1 and "device" in str(e.value)
    # a prepared dd_desc passes through unchanged
    d = dd.dd_desc(1024, 4, 1.0, dd.DD_C64, 4096, 1 << 20)
    assert dd._one_desc(d) is d
