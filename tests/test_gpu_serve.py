"""GPU tests of the request server: every result matches the FP64 oracle and
is bit-identical alone and in the mix; plain mode matches the plain
execution; admission respects the footprint budget; queue-full, too-large
and time-out statuses; batches overlap on the device under load."""
import numpy as np
import pytest

import siggen
from parity import assert_close, assert_same, spectrum_rms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def make_requests(seed, count, nmax=65536, extra=()):
    """Seeded (N, alpha, dtype code, numpy x) requests: N and alpha as the
    uneven mix, float32 real or complex64 input half and half."""
    import paper_2403_16665_amd as dd
    rng = np.random.default_rng(seed)
    pairs = [(n, a) for n, a in siggen.uneven_mix(rng, 4 * count) if n <= nmax][:count] + list(extra)
    out = []
    for i, (N, a) in enumerate(pairs):
        g = np.random.default_rng(seed * 1000 + i)
        if rng.random() < 0.5:
            out.append((N, a, dd.DD_F32, g.standard_normal(N).astype(np.float32)))
        else:
            out.append((N, a, dd.DD_C64, siggen.tones_complex(g, N, 1e-3)))
    return out


def device_buffers(reqs):
    import torch
    import paper_2403_16665_amd as dd
    xs, Xs = [], []
    for N, a, c, x in reqs:
        xs.append(torch.from_numpy(x).cuda())
        Xs.append(torch.zeros(a * N, dtype=dd.out_dtype(c), device="cuda"))
    torch.cuda.synchronize()  # the server's streams do not order after torch's
    return xs, Xs


def serve_all(server, reqs, xs, Xs):
    import paper_2403_16665_amd as dd
    tickets = [dd.dense_dft_submit(server, (N, a, N * 1e-3, c, xs[i], Xs[i])) for i, (N, a, c, _) in enumerate(reqs)]
    res = [dd.dense_dft_wait(server, t, 30_000_000) for t in tickets]
    assert all(r["status"] == 0 for r in res), res
    return res


def test_serve_mix_parity_alone_and_plain(oracle_mod):
    import torch
    import paper_2403_16665_amd as dd
    reqs = make_requests(31, 40, extra=[(24, 4), (3 * 2 ** 14, 3)])
    reqs.append((1024, 4, dd.DD_F64, siggen.tones_real(np.random.default_rng(8), 1024, 1e-3, 4)[0]))
    xs, Xs = device_buffers(reqs)
    srv = dd.dense_dft_server_create(hbm_budget_bytes=1 << 30, max_inflight=2, max_batch=8,
                                     flags=dd.DD_SERVE_DETERMINISTIC, batch_max_bins=-1)
    dd.dense_dft_server_pause(srv, True)      # queue everything, then let the batches form
    tickets = [dd.dense_dft_submit(srv, (N, a, N * 1e-3, c, xs[i], Xs[i])) for i, (N, a, c, _) in enumerate(reqs)]
    assert dd.dense_dft_poll(srv, tickets[0]) is None
    dd.dense_dft_server_pause(srv, False)
    res = [dd.dense_dft_wait(srv, t, 30_000_000) for t in tickets]
    assert all(r["status"] == 0 for r in res)
    st = dd.dense_dft_server_stats(srv)
    assert st["completed"] == len(reqs) and st["batches"] >= len(reqs) // 8
    assert st["max_batch_seen"] == 8 and st["fallback_requests"] >= 2  # N=24 and the float64 request
    assert st["peak_footprint"] <= 1 << 30
    mixed = [X.cpu().numpy() for X in Xs]
    rng = np.random.default_rng(5)
    for (N, a, c, x), X in zip(reqs, mixed):
        T = N * 1e-3
        bins = siggen.bin_subset(rng, a * N, 256)
        ref = oracle_mod.alpha_dft_bins(x, a, T, bins)
        kind = "f64" if c == dd.DD_F64 else "f32"
        full = None if len(bins) == a * N else spectrum_rms(x, T)
        assert_close(X[bins], ref, kind, f"served N={N} alpha={a} dtype={c}", full_rms=full)
    # each request alone (nothing else queued): bit-identical
    for i in range(0, len(reqs), 3):
        N, a, c, _ = reqs[i]
        X2 = torch.zeros_like(Xs[i])
        torch.cuda.synchronize()
        r = dd.dense_dft_wait(srv, dd.dense_dft_submit(srv, (N, a, N * 1e-3, c, xs[i], X2)), 30_000_000)
        assert r["status"] == 0 and r["batch_requests"] == 1
        assert np.array_equal(X2.cpu().numpy(), mixed[i]), f"request {i} differs alone vs in the mix"
    # and the plain per-signal path agrees within the FP32 bound
    for i in range(0, len(reqs), 4):
        N, a, c, _ = reqs[i]
        if c == dd.DD_F64:
            continue
        Xp = dd.alpha_dft(xs[i], a, N * 1e-3).cpu().numpy()
        assert_same(mixed[i], Xp, f"served vs plain, request {i}")
    dd.dense_dft_server_destroy(srv)


def test_serve_default_routing_alone_and_in_mix(oracle_mod):
    """Default server: a request alone runs as a plain execution, large ones
    always do, the rest batch; each result is the same alone and in the mix
    within the FP32 bound, and matches the oracle."""
    import torch
    import paper_2403_16665_amd as dd
    reqs = make_requests(34, 24, nmax=262144, extra=[(262144, 16), (131072, 8)])
    xs, Xs = device_buffers(reqs)
    srv = dd.dense_dft_server_create(hbm_budget_bytes=2 << 30, max_batch=32)
    dd.dense_dft_server_pause(srv, True)
    tickets = [dd.dense_dft_submit(srv, (N, a, N * 1e-3, c, xs[i], Xs[i])) for i, (N, a, c, _) in enumerate(reqs)]
    dd.dense_dft_server_pause(srv, False)
    res = [dd.dense_dft_wait(srv, t, 30_000_000) for t in tickets]
    assert all(r["status"] == 0 for r in res)
    st = dd.dense_dft_server_stats(srv)
    big = sum(1 for N, a, _, _ in reqs if a * N > (1 << 20))
    assert big >= 1 and st["fallback_requests"] >= big and st["kernel_requests"] >= 1
    mixed = [X.cpu().numpy() for X in Xs]
    rng = np.random.default_rng(9)
    for i, (N, a, c, x) in enumerate(reqs):
        X2 = torch.zeros_like(Xs[i])
        torch.cuda.synchronize()
        r = dd.dense_dft_wait(srv, dd.dense_dft_submit(srv, (N, a, N * 1e-3, c, xs[i], X2)), 30_000_000)
        assert r["status"] == 0 and r["batch_requests"] == 1
        assert_same(mixed[i], X2.cpu().numpy(), f"request {i} in the mix vs alone")
        if i % 3 == 0:
            bins = siggen.bin_subset(rng, a * N, 128)
            assert_close(mixed[i][bins], oracle_mod.alpha_dft_bins(x, a, N * 1e-3, bins), "f32",
                         f"routed N={N} alpha={a}", full_rms=spectrum_rms(x, N * 1e-3))
    dd.dense_dft_server_destroy(srv)


def test_serve_plain_mode_matches_plain_exec():
    """Plain mode, with a scheduler that sleeps as soon as it is idle
    (spin_us = -1): every request is one plain execution, bit-identical to
    the plain transform."""
    import torch
    import paper_2403_16665_amd as dd
    reqs = make_requests(32, 12)
    xs, Xs = device_buffers(reqs)
    srv = dd.dense_dft_server_create(mode=dd.DD_SERVE_PLAIN, hbm_budget_bytes=1 << 30, spin_us=-1)
    res = serve_all(srv, reqs, xs, Xs)
    assert all(r["batch_requests"] == 1 for r in res)
    st = dd.dense_dft_server_stats(srv)
    assert st["kernel_requests"] == 0 and st["fallback_requests"] == len(reqs) and st["batches"] == len(reqs)
    for i, (N, a, c, _) in enumerate(reqs):
        ref = dd.alpha_dft(xs[i], a, N * 1e-3)
        torch.cuda.synchronize()
        assert torch.equal(ref, Xs[i]), f"plain-mode request {i} differs from the plain execution"
    dd.dense_dft_server_destroy(srv)


def test_serve_status_codes():
    import torch
    import paper_2403_16665_amd as dd
    x = torch.zeros(65536, dtype=torch.complex64, device="cuda")
    X = torch.zeros(8 * 65536, dtype=torch.complex64, device="cuda")
    small = dd.dense_dft_server_create(hbm_budget_bytes=1 << 20, max_queue=2)
    with pytest.raises(dd.DenseDFTError) as e:
        dd.dense_dft_submit(small, (65536, 8, 65.536, dd.DD_C64, x, X))   # 4.5 MiB > 1 MiB budget
    assert e.value.status == dd.DD_ERR_TOO_LARGE
    with pytest.raises(dd.DenseDFTError) as e:
        dd.dense_dft_submit(small, (65536, 8, 65.536, dd.DD_C64, x, x))   # x and X overlap
    assert e.value.status == 1
    xs = torch.zeros(256, dtype=torch.complex64, device="cuda")
    Xa = torch.zeros(3, 4 * 256, dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()
    dd.dense_dft_server_pause(small, True)
    t1 = dd.dense_dft_submit(small, (256, 4, 0.256, dd.DD_C64, xs, Xa[0]))
    t2 = dd.dense_dft_submit(small, (256, 4, 0.256, dd.DD_C64, xs, Xa[1]))
    with pytest.raises(dd.DenseDFTError) as e:
        dd.dense_dft_submit(small, (256, 4, 0.256, dd.DD_C64, xs, Xa[2]))  # max_queue = 2
    assert e.value.status == dd.DD_ERR_BUSY
    with pytest.raises(dd.DenseDFTError) as e:
        dd.dense_dft_wait(small, t1, 1000)                                  # held: times out
    assert e.value.status == dd.DD_ERR_TIMEOUT
    assert dd.dense_dft_poll(small, t2) is None
    dd.dense_dft_server_pause(small, False)
    assert dd.dense_dft_wait(small, t1, 10_000_000)["status"] == 0
    assert dd.dense_dft_wait(small, t2, 10_000_000)["status"] == 0
    with pytest.raises(dd.DenseDFTError) as e:
        dd.dense_dft_poll(small, t1)                                        # retired ticket
    assert e.value.status == 1
    dd.dense_dft_server_destroy(small)


def test_serve_batches_overlap_under_load():
    """Open-loop arrivals faster than one batch completes: later requests are
    admitted while earlier batches run, the in-flight footprint stays within
    the budget, and results match a plain execution."""
    import time
    import torch
    import paper_2403_16665_amd as dd
    rng = np.random.default_rng(77)
    N, a = 65536, 8
    base = [siggen.tones_complex(np.random.default_rng(i), N, 1e-3) for i in range(4)]
    xs = [torch.from_numpy(b).cuda() for b in base]
    count = 160
    Xs = torch.zeros(count, a * N, dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()
    budget = 48 << 20   # about five requests' footprint
    srv = dd.dense_dft_server_create(hbm_budget_bytes=budget, max_inflight=2, max_batch=64)
    dd.dense_dft_server_warm(srv, N, a, N * 1e-3, dd.DD_C64)
    arrivals = siggen.poisson_arrivals(rng, 20000.0, count)
    t0 = dd.dense_dft_clock_ns() + 1_000_000
    tickets = []
    for i in range(count):
        due = t0 + int(arrivals[i] * 1e9)
        while dd.dense_dft_clock_ns() < due:
            pass
        tickets.append(dd.dense_dft_submit(srv, (N, a, N * 1e-3, dd.DD_C64, xs[i % 4], Xs[i]), due))
    res = [dd.dense_dft_wait(srv, t, 30_000_000) for t in tickets]
    st = dd.dense_dft_server_stats(srv)
    dd.dense_dft_server_destroy(srv)
    assert all(r["status"] == 0 for r in res)
    assert st["peak_footprint"] <= budget and st["max_batch_seen"] > 1
    starts = sorted((r["t_start_ns"], r["t_done_ns"]) for r in res)
    overlapped = any(s2 < d1 for (s1, d1), (s2, d2) in zip(starts, starts[1:]) if s2 > s1)
    assert overlapped, "no batch was launched while another was on the device"
    lat = np.array([r["t_done_ns"] - r["t_arrival_ns"] for r in res]) / 1e6
    assert np.all(lat > 0)
    ref = [dd.alpha_dft(x, a, N * 1e-3) for x in xs]
    torch.cuda.synchronize()
    for i in range(0, count, 7):
        assert_same(Xs[i].cpu().numpy(), ref[i % 4].cpu().numpy(), f"request {i}")


def test_serve_caller_stream_and_fp32_twiddles(oracle_mod):
    """A server whose slots share the caller's stream, with the FP32-twiddle
    variant: results match the oracle, and match a plain execution made with
    the same twiddle flag."""
    import torch
    import paper_2403_16665_amd as dd
    reqs = make_requests(36, 10, nmax=65536)
    xs, Xs = device_buffers(reqs)
    stream = torch.cuda.Stream()
    srv = dd.dense_dft_server_create(hbm_budget_bytes=1 << 30, flags=dd.DD_TWIDDLE_FP32,
                                     hip_stream=stream.cuda_stream)
    dd.dense_dft_server_pause(srv, True)
    tickets = [dd.dense_dft_submit(srv, (N, a, N * 1e-3, c, xs[i], Xs[i])) for i, (N, a, c, _) in enumerate(reqs)]
    dd.dense_dft_server_pause(srv, False)
    res = [dd.dense_dft_wait(srv, t, 30_000_000) for t in tickets]
    assert all(r["status"] == 0 for r in res)
    dd.dense_dft_server_destroy(srv)
    rng = np.random.default_rng(13)
    for i, (N, a, c, x) in enumerate(reqs):
        got = Xs[i].cpu().numpy()
        bins = siggen.bin_subset(rng, a * N, 128)
        assert_close(got[bins], oracle_mod.alpha_dft_bins(x, a, N * 1e-3, bins), "f32",
                     f"fp32-twiddle server N={N} alpha={a}", full_rms=spectrum_rms(x, N * 1e-3))
        ref = dd.alpha_dft(xs[i], a, N * 1e-3, flags=dd.DD_TWIDDLE_FP32).cpu().numpy()
        assert_same(got, ref, f"fp32-twiddle served vs plain, request {i}")


def test_class_schedule_survives_a_tuning_change(oracle_mod, tmp_path):
    """A class's schedule is fixed when the server first makes its tables: a
    later change of the tuning table (here: the two-pass entry the class was
    first served with is cleared, so the class now classifies as one pass)
    must not change what the server's kernel items use (their scratch
    included).  Both requests are checked against the oracle."""
    import paper_2403_16665_amd as dd
    N, alpha = 1024, 4
    db = tmp_path / "two_pass.txt"
    db.write_text(f"batch {N} {alpha} 2 32 32 1.0\n")
    dd.dense_dft_tune_clear()
    dd.dense_dft_tune_load(str(db))
    try:
        srv = dd.dense_dft_server_create(hbm_budget_bytes=1 << 28, max_inflight=1, max_batch=4,
                                         flags=dd.DD_SERVE_DETERMINISTIC, batch_max_bins=-1)
        reqs = make_requests(77, 0, extra=[(N, alpha), (N, alpha)])
        xs, Xs = device_buffers(reqs)
        serve_all(srv, reqs[:1], xs[:1], Xs[:1])        # class tables made with the two-pass entry
        dd.dense_dft_tune_clear()                       # the class now classifies as one pass
        serve_all(srv, reqs[1:], xs[1:], Xs[1:])
        st = dd.dense_dft_server_stats(srv)
        assert st["kernel_requests"] == 2 and st["classes"] == 1
        dd.dense_dft_server_destroy(srv)
    finally:
        dd.dense_dft_tune_clear()
    for (n, a, c, x), X in zip(reqs, Xs):
        ref = oracle_mod.alpha_dft(x, a, n * 1e-3)
        assert_close(X.cpu().numpy(), ref, "f32", f"N={n} alpha={a}")


def test_plain_workspace_within_the_servers_reservation():
    """The server reserves, for a request of alpha N bins, the spectrum's
    bytes plus 1/8 when the spectrum takes at least 64 KiB (the most that
    padded scratch rows add); a plain execution of one signal, which any
    request may become, needs no more under any schedule.  Also pins that the
    rows of long row groups are padded (2^22 x alpha 16) and short ones not."""
    import paper_2403_16665_amd as dd
    shapes = [(262144, 16), (262144, 2), (131072, 8), (65536, 8), (4194304, 16), (1 << 20, 4), (3 * 4096, 16)]
    for N, a in shapes:
        for code, elem in ((dd.DD_C64, 8), (dd.DD_F32, 8), (dd.DD_C128, 16)):
            spec = a * N * elem
            bound = spec + spec // 8 if spec >= 64 * 1024 else spec
            for sc in dd.dense_dft_sched_candidates(N, a, 1, code):
                if sc.passes != 2:
                    continue
                try:
                    plan = dd.dense_dft_plan_sched(N, a, N * 1e-3, 1, code, sc, dd.DD_NO_WORKSPACE)
                except dd.DenseDFTError:
                    continue   # a split the kernels of this precision do not hold
                ws = dd.dense_dft_workspace_size(plan)
                assert spec <= ws <= bound, (N, a, code, sc.N1, sc.N2, ws, bound)
                if (N, a, code) == (4194304, 16, dd.DD_C64) and sc.N2 == 1024:
                    assert ws == a * sc.N1 * (sc.N2 + 64) * 8   # rows padded by 512 bytes
                if (N, a, elem) == (65536, 8, 8) and sc.N2 <= 512:
                    assert ws == spec                          # short row groups unpadded
                dd.dense_dft_destroy(plan)
