"""Parity at the benchmark's full sizes, in the configurations bench.py times,
on sampled outputs the oracle evaluates one by one: the persistent batch of
the 1000-signal uneven mix, and a stream of requests through the server at
400k requests/s (float32 real and complex64 inputs, half each)."""
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


def test_uneven_1000_batch_sampled(oracle_mod):
    """The uneven workload of bench.py: 1000 complex64 signals, one batch
    execution; 40 seeded signals checked on 64 seeded bins each against the
    oracle, 5 of them over the whole spectrum against plain executions."""
    import torch
    import paper_2403_16665_amd as dd
    dt = 1e-3
    mix = siggen.uneven_mix(siggen.rngs(3, 1)[0], 1000)
    gens = siggen.rngs(4, len(mix))
    xs = [torch.from_numpy(siggen.tones_complex(g, N, dt)).cuda() for g, (N, a) in zip(gens, mix)]
    Xs = [torch.zeros(a * N, dtype=torch.complex64, device="cuda") for (N, a) in mix]
    b = dd.dense_dft_batch_plan([(N, a, N * dt, dd.DD_C64, xs[i], Xs[i]) for i, (N, a) in enumerate(mix)])
    dd.dense_dft_batch_exec(b)
    torch.cuda.synchronize()
    assert dd.dense_dft_batch_status(b) == 0
    rng = np.random.default_rng(77)
    picks = sorted(rng.choice(len(mix), size=40, replace=False))
    for i in picks:
        N, a = mix[i]
        x = xs[i].cpu().numpy()
        bins = siggen.bin_subset(rng, a * N, 64)
        got = Xs[i].cpu().numpy()[bins]
        assert_close(got, oracle_mod.alpha_dft_bins(x, a, N * dt, bins), "f32", f"signal {i} N={N} alpha={a}",
                     full_rms=spectrum_rms(x, N * dt))
    for i in picks[:5]:
        N, a = mix[i]
        ref = dd.alpha_dft(xs[i], a, N * dt)
        torch.cuda.synchronize()
        assert_same(Xs[i].cpu().numpy(), ref.cpu().numpy(), f"batch vs plain, signal {i}")


def test_serving_stream_sampled(oracle_mod):
    """The serving workload of bench.py at 400k requests/s, 2000 requests
    with pre-drawn Poisson arrivals through a default server: every request
    completes, and 40 seeded requests match the oracle on 64 seeded bins."""
    import torch
    import paper_2403_16665_amd as dd
    dt = 1e-3
    count = 2000
    rng = siggen.rngs(5, 1)[0]
    mix = siggen.uneven_mix(rng, count)
    codes = [dd.DD_F32 if u < 0.5 else dd.DD_C64 for u in rng.random(count)]
    inputs = {}
    kinds = sorted(set((N, c) for (N, _), c in zip(mix, codes)))
    for g, (N, c) in zip(siggen.rngs(6, len(kinds)), kinds):
        if c == dd.DD_F32:
            inputs[(N, c)] = torch.from_numpy(siggen.tones_real(g, N, dt, 1)[0].astype(np.float32)).cuda()
        else:
            inputs[(N, c)] = torch.from_numpy(siggen.tones_complex(g, N, dt)).cuda()
    offs = np.concatenate([[0], np.cumsum([a * N for N, a in mix])])
    arena = torch.zeros(int(offs[-1]), dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()
    descs = [(N, a, N * dt, c, inputs[(N, c)], arena[int(offs[i]):int(offs[i + 1])])
             for i, ((N, a), c) in enumerate(zip(mix, codes))]
    srv = dd.dense_dft_server_create(hbm_budget_bytes=16 << 30)
    arr = siggen.poisson_arrivals(np.random.default_rng(100), 400000.0, count)
    t0 = dd.dense_dft_clock_ns() + 2_000_000
    tickets = dd.dense_dft_submit_many_at(srv, descs, [t0 + int(s * 1e9) for s in arr])
    res = [dd.dense_dft_wait(srv, t, 120_000_000) for t in tickets]
    assert all(r["status"] == 0 for r in res)
    st = dd.dense_dft_server_stats(srv)
    assert st["completed"] == count and st["max_batch_seen"] > 1
    dd.dense_dft_server_destroy(srv)
    check = np.random.default_rng(78)
    for i in sorted(check.choice(count, size=40, replace=False)):
        (N, a), c = mix[i], codes[i]
        x = inputs[(N, c)].cpu().numpy()
        bins = siggen.bin_subset(check, a * N, 64)
        got = arena[int(offs[i]):int(offs[i + 1])].cpu().numpy()[bins]
        assert_close(got, oracle_mod.alpha_dft_bins(x, a, N * dt, bins), "f32",
                     f"request {i} N={N} alpha={a} dtype={c}", full_rms=spectrum_rms(x, N * dt))
