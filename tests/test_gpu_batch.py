"""GPU tests of the persistent batched path (many signals of uneven N and alpha
in one launch): parity with the FP64 oracle, identical results alone and in a
mix, agreement with the plain per-signal path, HIP-graph capture and replay."""
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


def make_mix(seed, count, nmax=16384, extra=()):
    """(N, alpha, dtype code, numpy x) for a seeded uneven mix."""
    import paper_2403_16665_amd as dd
    rng = np.random.default_rng(seed)
    pairs = [(n, a) for n, a in siggen.uneven_mix(rng, 4 * count) if n <= nmax][:count]
    pairs += list(extra)
    out = []
    for i, (N, a) in enumerate(pairs):
        g = np.random.default_rng(seed * 1000 + i)
        if i % 3 == 2:
            x = g.standard_normal(N).astype(np.float32)
            out.append((N, a, dd.DD_F32, x))
        else:
            x = siggen.tones_complex(g, N, 1e-3)
            out.append((N, a, dd.DD_C64, x))
    return out


def run_batch(sigs, T_of=lambda N: N * 1e-3):
    import torch
    import paper_2403_16665_amd as dd
    xs = [torch.from_numpy(x).cuda() for (_, _, _, x) in sigs]
    Xs = [torch.empty(a * N, dtype=torch.complex64, device="cuda") for (N, a, _, _) in sigs]
    descs = [(N, a, T_of(N), c, xs[i], Xs[i]) for i, (N, a, c, _) in enumerate(sigs)]
    b = dd.dense_dft_batch_plan(descs)
    dd.dense_dft_batch_exec(b)
    torch.cuda.synchronize()
    assert dd.dense_dft_batch_status(b) == 0
    return b, [X.cpu().numpy() for X in Xs]


def check_against_oracle(oracle_mod, sigs, outs, nbins=256, T_of=lambda N: N * 1e-3):
    rng = np.random.default_rng(77)
    for (N, a, c, x), X in zip(sigs, outs):
        T = T_of(N)
        bins = siggen.bin_subset(rng, a * N, nbins)
        ref = oracle_mod.alpha_dft_bins(x, a, T, bins)
        full = None if len(bins) == a * N else spectrum_rms(x, T)
        assert_close(X[bins], ref, "f32", f"N={N} alpha={a} dtype={c}", full_rms=full)


def test_batch_mixed_parity_alone_and_plain(oracle_mod):
    import torch
    import paper_2403_16665_amd as dd
    sigs = make_mix(5, 36, extra=[(65536, 8), (3 * 2 ** 15, 3), (5 * 2 ** 14, 16), (24, 4), (1 << 18, 2)])
    b, outs = run_batch(sigs)
    tasks, grid, scratch, fb = dd.dense_dft_batch_info(b)
    assert tasks > len(sigs) and grid >= 1
    assert fb >= 1  # N = 24 is not compiled into the batch kernel: plain fallback
    check_against_oracle(oracle_mod, sigs, outs)
    # each signal alone (a batch of one) gives bit-identical output
    for i in range(0, len(sigs), 4):
        _, alone = run_batch([sigs[i]])
        assert np.array_equal(alone[0], outs[i]), f"signal {i} differs alone vs in the mix"
    # and agrees with the plain per-signal path
    for i in range(0, len(sigs), 5):
        N, a, c, x = sigs[i]
        Xp = dd.alpha_dft(torch.from_numpy(x).cuda(), a, N * 1e-3).cpu().numpy()
        assert_same(outs[i], Xp, f"batch vs plain, signal {i}")


def test_batch_real_and_complex_same_signal():
    """A real float32 signal and the same samples as complex64 give the same spectrum."""
    g = np.random.default_rng(3)
    xr = g.standard_normal(4096).astype(np.float32)
    import paper_2403_16665_amd as dd
    sigs = [(4096, 8, dd.DD_F32, xr), (4096, 8, dd.DD_C64, xr.astype(np.complex64))]
    _, outs = run_batch(sigs)
    assert np.array_equal(outs[0], outs[1])


def test_batch_graph_replay(oracle_mod):
    """Capture one batch execution in a HIP graph, replay it with new input
    samples and with new buffers (descriptor table refreshed at replay), and
    check every replay against an eager execution."""
    import torch
    import paper_2403_16665_amd as dd
    sigs = make_mix(11, 12, nmax=65536)
    xs = [torch.from_numpy(x).cuda() for (_, _, _, x) in sigs]
    Xs = [torch.zeros(a * N, dtype=torch.complex64, device="cuda") for (N, a, _, _) in sigs]
    descs = [(N, a, N * 1e-3, c, xs[i], Xs[i]) for i, (N, a, c, _) in enumerate(sigs)]
    b = dd.dense_dft_batch_plan(descs)
    # eager reference of the same inputs
    ref_X = [torch.zeros_like(X) for X in Xs]
    ref_b = dd.dense_dft_batch_plan([(N, a, T, c, x, R) for (N, a, T, c, x, _), R in zip(descs, ref_X)])
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        dd.dense_dft_batch_exec(b, stream=torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        gen = np.random.default_rng(100 + rep)
        for x in xs:  # new samples in the same buffers
            x.copy_(torch.from_numpy(
                (gen.standard_normal(x.shape[0]) * (1 + 1j)).astype(np.complex64)
                if x.dtype == torch.complex64 else gen.standard_normal(x.shape[0]).astype(np.float32)).cuda())
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        dd.dense_dft_batch_exec(ref_b)
        torch.cuda.synchronize()
        for X, R in zip(Xs, ref_X):
            assert torch.equal(X, R), f"replay {rep} differs from eager"
    assert dd.dense_dft_batch_status(b) == 0
    # new output buffers, same shapes: the replay writes into them
    Xs2 = [torch.zeros_like(X) for X in Xs]
    dd.dense_dft_batch_set_buffers(b, [(N, a, T, c, x, X2) for (N, a, T, c, x, _), X2 in zip(descs, Xs2)])
    g.replay()
    torch.cuda.synchronize()
    for X2, R in zip(Xs2, ref_X):
        assert torch.equal(X2, R)
    # shape mismatch is rejected
    bad = list(descs)
    N, a, T, c, x, X = bad[0]
    bad[0] = (N, a + 1, T, c, x, X)
    with pytest.raises(dd.DenseDFTError):
        dd.dense_dft_batch_set_buffers(b, bad)


def test_exec_many_and_fp64_fallback(oracle_mod):
    import torch
    import paper_2403_16665_amd as dd
    g = np.random.default_rng(21)
    x1 = siggen.tones_complex(g, 8192, 1e-3)
    x2, _ = siggen.tones_real(g, 1024, 1e-3, 4)          # float64: plain fallback
    X1 = torch.empty(4 * 8192, dtype=torch.complex64, device="cuda")
    X2 = torch.empty(4 * 1024, dtype=torch.complex128, device="cuda")
    d1, d2 = torch.from_numpy(x1).cuda(), torch.from_numpy(x2).cuda()
    dd.dense_dft_exec_many([(8192, 4, 8.192, dd.DD_C64, d1, X1), (1024, 4, 1.024, dd.DD_F64, d2, X2)])
    bins = siggen.bin_subset(g, 4 * 8192, 512)
    assert_close(X1.cpu().numpy()[bins], oracle_mod.alpha_dft_bins(x1, 4, 8.192, bins), "f32", "c64",
                 full_rms=spectrum_rms(x1, 8.192))
    assert_close(X2.cpu().numpy(), oracle_mod.alpha_dft(x2, 4, 1.024), "f64", "f64 fallback")


def test_batch_fp32_twiddles(oracle_mod):
    import torch
    import paper_2403_16665_amd as dd
    sigs = make_mix(17, 12, nmax=65536)
    xs = [torch.from_numpy(x).cuda() for (_, _, _, x) in sigs]
    Xs = [torch.empty(a * N, dtype=torch.complex64, device="cuda") for (N, a, _, _) in sigs]
    b = dd.dense_dft_batch_plan([(N, a, N * 1e-3, c, xs[i], Xs[i]) for i, (N, a, c, _) in enumerate(sigs)],
                                flags=dd.DD_TWIDDLE_FP32)
    dd.dense_dft_batch_exec(b)
    torch.cuda.synchronize()
    check_against_oracle(oracle_mod, sigs, [X.cpu().numpy() for X in Xs])
