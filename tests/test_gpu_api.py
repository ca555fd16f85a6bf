"""Entry points around the transform: per-launch profiling of a plan and the
server's open-loop submission of a pre-drawn arrival schedule."""
import numpy as np
import pytest

import siggen
from parity import assert_close, spectrum_rms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_profile_records_every_launch():
    """Two passes over two chunks, then the inverse: one record per kernel
    launch in enqueue order, each with a positive duration; a one-pass plan
    records kind `single`; max_launches bounds what is recorded."""
    import torch
    import paper_2403_16665_amd as dd
    N, alpha, batch = 65536, 8, 35
    sc = dd.make_sched(2, N1=256, N2=256, jgroup=8, chunk=32)
    plan = dd.dense_dft_plan_sched(N, alpha, 1.0, batch, dd.DD_C64, sc)
    x = torch.randn(batch, N, dtype=torch.complex64, device="cuda")
    X = torch.empty(batch, alpha * N, dtype=torch.complex64, device="cuda")
    back = torch.empty_like(x)
    dd.dense_dft_profile_begin(plan, 64)
    dd.dense_dft_exec(plan, x, X)
    dd.dense_dft_exec_inverse(plan, X, back)
    rec = dd.dense_dft_profile_end(plan)
    assert [k for k, _ in rec] == ["pass1", "pass2", "pass1", "pass2",
                                   "inverse_passA", "inverse_passB", "inverse_passA", "inverse_passB"]
    assert all(ms > 0 for _, ms in rec)
    # profiling is off again: a further execution records nothing
    dd.dense_dft_exec(plan, x, X)
    dd.dense_dft_profile_begin(plan, 1)
    dd.dense_dft_exec(plan, x, X)
    assert [k for k, _ in dd.dense_dft_profile_end(plan)] == ["pass1"]
    one = dd.dense_dft_plan(1024, 4, 1.0, 3, dd.DD_F32)
    xr = torch.randn(3, 1024, device="cuda")
    dd.dense_dft_profile_begin(one, 8)
    dd.dense_dft_exec(one, xr, torch.empty(3, 4096, dtype=torch.complex64, device="cuda"))
    rec = dd.dense_dft_profile_end(one)
    assert [k for k, _ in rec] == ["single"] and rec[0][1] > 0


def test_submit_many_at_open_loop(oracle_mod):
    """Requests queued at pre-drawn host times: each is stamped with its
    scheduled arrival, starts no earlier and finishes after it starts, and
    its spectrum matches the oracle.  Non-decreasing times are required."""
    import torch
    import paper_2403_16665_amd as dd
    rng = np.random.default_rng(12)
    shapes = [(1024, 4), (4096, 8), (65536, 2), (3 * 2 ** 10, 3), (262144, 16), (256, 16)]
    xs, Xs, descs = [], [], []
    for i, (N, a) in enumerate(shapes):
        x = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64) if i % 2 else \
            rng.standard_normal(N).astype(np.float32)
        xs.append(torch.from_numpy(x).cuda())
        Xs.append(torch.zeros(a * N, dtype=torch.complex64, device="cuda"))
        descs.append((N, a, N * 1e-3, dd.DD_C64 if i % 2 else dd.DD_F32, xs[-1], Xs[-1]))
    torch.cuda.synchronize()
    srv = dd.dense_dft_server_create(hbm_budget_bytes=1 << 30)
    t0 = dd.dense_dft_clock_ns() + 1_000_000
    due = [t0 + i * 200_000 for i in range(len(descs))]
    tickets = dd.dense_dft_submit_many_at(srv, descs, due)
    res = [dd.dense_dft_wait(srv, t, 30_000_000) for t in tickets]
    for r, d in zip(res, due):
        assert r["status"] == 0
        assert r["t_arrival_ns"] == d and r["t_start_ns"] >= d and r["t_done_ns"] >= r["t_start_ns"]
    for (N, a), x, X in zip(shapes, xs, Xs):
        xn = x.cpu().numpy()
        bins = siggen.bin_subset(rng, a * N, 256)
        full = None if len(bins) == a * N else spectrum_rms(xn, N * 1e-3)
        assert_close(X.cpu().numpy()[bins], oracle_mod.alpha_dft_bins(xn, a, N * 1e-3, bins), "f32",
                     f"N={N} alpha={a}", full_rms=full)
    # a decreasing time is refused at that request; the ones before it are queued
    now = dd.dense_dft_clock_ns()
    with pytest.raises(dd.DenseDFTError, match="queued 1 of 2"):
        dd.dense_dft_submit_many_at(srv, descs[:2], [now + 100_000, now])
    dd.dense_dft_server_destroy(srv)   # drains the queued request


def test_binding_rejects_mismatched_device_tensors():
    """Device tensors of the wrong dtype, too short, strided, or a workspace
    smaller than the plan's: DD_ERR_INVALID from the binding, no launch."""
    import torch
    import paper_2403_16665_amd as dd
    plan = dd.dense_dft_plan(65536, 8, 1.0, 2, dd.DD_C64)
    x = torch.zeros(2, 65536, dtype=torch.complex64, device="cuda")
    X = torch.zeros(2, 8 * 65536, dtype=torch.complex64, device="cuda")
    ws_need = dd.dense_dft_workspace_size(plan)
    assert ws_need > 0
    bad = [lambda: dd.dense_dft_exec(plan, x.to(torch.complex128), X),
           lambda: dd.dense_dft_exec(plan, x, X[:, :-1]),
           lambda: dd.dense_dft_exec(plan, x[:1], X),
           lambda: dd.dense_dft_exec(plan, torch.zeros(65536, 2, dtype=torch.complex64, device="cuda").t(), X),
           lambda: dd.dense_dft_exec(plan, x, X, workspace=torch.empty(ws_need - 1, dtype=torch.uint8,
                                                                         device="cuda")),
           lambda: dd.dense_dft_exec_inverse(plan, X[:, :-8], x),
           lambda: dd.dense_dft_exec_inverse(plan, X, x.real.contiguous())]
    for i, call in enumerate(bad):
        with pytest.raises(dd.DenseDFTError) as e:
            call()
        assert e.value.status == 1, i
    # the exact buffers and a workspace of exactly the reported size are accepted
    dd.dense_dft_exec(plan, x, X, workspace=torch.empty(ws_need, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()


def test_scale_at_the_ends_of_float_range(oracle_mod):
    """A tiny T/N (1e-30) and a huge T (1e38) in float: the forward transform
    matches the oracle at both.  At T = 1e38 and alpha = 2, 1/(alpha T) is
    below float's normal range, so the inverse is refused
    (DD_ERR_UNSUPPORTED) instead of returning flushed zeros."""
    import torch
    import paper_2403_16665_amd as dd
    N, alpha = 64, 2
    rng = np.random.default_rng(8)
    x = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
    xd = torch.from_numpy(x).cuda()
    for T in (N * 1e-30, 1e38):
        X = dd.alpha_dft(xd, alpha, T).cpu().numpy()
        assert_close(X, oracle_mod.alpha_dft(x, alpha, T), "f32", f"T={T}")
    plan = dd.dense_dft_plan(N, alpha, 1e38, 1, dd.DD_C64)
    X = plan.exec(xd.reshape(1, N))
    with pytest.raises(dd.DenseDFTError) as e:
        plan.exec_inverse(X)
    assert e.value.status == 2
    torch.cuda.synchronize()
