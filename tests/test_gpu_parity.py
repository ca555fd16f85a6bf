"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Inputs are seeded (siggen); the oracle sees the exact stored samples.  Small
and medium sizes compare every output bin; full-size workloads compare a
seeded random subset of bins (the oracle evaluates bins one at a time).
"""
import os

import numpy as np
import pytest

import siggen
from parity import assert_close, gpu_alpha_dft, rel_l2, spectrum_rms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def cplx(rng, shape, dtype=np.complex64):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dtype)


SINGLE_N = [1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192,
            256, 320, 384, 512, 640, 768, 1024, 1280, 1536, 2048, 2560, 3072, 4096]


@pytest.mark.parametrize("N", SINGLE_N)
@pytest.mark.parametrize("alpha", [1, 2, 3, 8])
def test_c64_full_spectrum(oracle_mod, N, alpha):
    """Every bin of every signal of a small ragged batch (covers one-pass and,
    for large alpha*N, two-pass schedules)."""
    rng = np.random.default_rng(N * 100 + alpha)
    batch = 3
    x = cplx(rng, (batch, N))
    T = 0.001 * N
    X = gpu_alpha_dft(x, alpha, T)
    assert X.shape == (batch, alpha * N)
    for b in range(batch):
        ref = oracle_mod.alpha_dft(x[b], alpha, T)
        assert_close(X[b], ref, "f32", f"N={N} alpha={alpha} sig={b}")


@pytest.mark.parametrize("N,alpha", [(256, 16), (4096, 4), (8192, 2), (16384, 3),
                                     (48, 256), (3 * 2 ** 12, 5), (5 * 2 ** 11, 4)])
def test_c64_two_pass_full_spectrum(oracle_mod, N, alpha):
    rng = np.random.default_rng(N + alpha)
    x = cplx(rng, (2, N))
    T = 1.5
    X = gpu_alpha_dft(x, alpha, T)
    for b in range(2):
        ref = oracle_mod.alpha_dft(x[b], alpha, T)
        assert_close(X[b], ref, "f32", f"N={N} alpha={alpha} sig={b}")


@pytest.mark.parametrize("dtype,kind", [(np.float32, "f32"), (np.float64, "f64"),
                                        (np.complex128, "f64")])
@pytest.mark.parametrize("N,alpha", [(1, 4), (12, 3), (1024, 4), (640, 16), (65536, 2)])
def test_dtypes(oracle_mod, dtype, kind, N, alpha):
    rng = np.random.default_rng(7 * N + alpha)
    if np.issubdtype(dtype, np.complexfloating):
        x = cplx(rng, (2, N), dtype)
    else:
        x = rng.standard_normal((2, N)).astype(dtype)
    T = 2.0
    X = gpu_alpha_dft(x, alpha, T)
    assert X.dtype == (np.complex64 if kind == "f32" else np.complex128)
    M = alpha * N
    bins = siggen.bin_subset(rng, M, 4096)
    for b in range(2):
        ref = oracle_mod.alpha_dft_bins(x[b], alpha, T, bins)
        assert_close(X[b][bins], ref, kind, f"{dtype.__name__} N={N} alpha={alpha}",
                     full_rms=spectrum_rms(x[b], T) if M > len(bins) else None)
        if not np.issubdtype(dtype, np.complexfloating) and M > 1:
            # real input: Hermitian symmetry of the full GPU spectrum
            mirror = X[b][(M - np.arange(M)) % M]
            assert_close(mirror, np.conj(X[b]), kind, f"Hermitian symmetry N={N} alpha={alpha}")


def test_plain_float64_real_workload(oracle_mod):
    """One real float64 signal, N = 1024 at dt = 1e-3 s (T = 1.024 s), alpha = 4:
    three off-bin sinusoids plus noise; all 4096 bins."""
    x, _ = siggen.tones_real(siggen.rngs(0, 1)[0], 1024, 1e-3, 4)
    X = gpu_alpha_dft(x[None, :], 4, 1.024)[0]
    ref = oracle_mod.alpha_dft(x, 4, 1.024)
    assert_close(X, ref, "f64", "real f64 N=1024 alpha=4")


def test_batch_c64_full_size_sampled(oracle_mod):
    """256 complex64 signals, N = 65536, alpha = 8 (524288 bins each), in the
    launch configuration the benchmark times; a seeded subset of bins of a
    spread of signals, plus exact structure checks on every signal."""
    import torch
    import paper_2403_16665_amd as dd
    N, alpha, batch, dt = 65536, 8, 256, 1e-3
    T = N * dt
    gens = siggen.rngs(1, batch)
    x = np.stack([siggen.tones_complex(g, N, dt) for g in gens])
    xd = torch.from_numpy(x).cuda()
    plan = dd.dense_dft_plan(N, alpha, T, batch, dd.DD_C64)
    Xd = torch.empty((batch, alpha * N), dtype=torch.complex64, device="cuda")
    dd.dense_dft_exec(plan, xd, Xd)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for b in [0, 1, 31, 32, 127, 200, 255]:
        bins = siggen.bin_subset(rng, alpha * N, 256)
        got = Xd[b].cpu().numpy()[bins]
        ref = oracle_mod.alpha_dft_bins(x[b], alpha, T, bins)
        assert_close(got, ref, "f32", f"signal {b}", full_rms=spectrum_rms(x[b], T))
    # every signal: X_{alpha k} is the coarse spectrum, and Parseval (eq. (8))
    Xc = Xd[:, ::alpha].to(torch.complex128)
    ref_coarse = torch.fft.fft(xd.to(torch.complex128), dim=1) * (T / N)
    err = (Xc - ref_coarse).abs().pow(2).sum(1).sqrt() / ref_coarse.abs().pow(2).sum(1).sqrt()
    assert float(err.max()) < 1e-5
    e_out = Xd.to(torch.complex128).abs().pow(2).sum(1)
    e_in = xd.to(torch.complex128).abs().pow(2).sum(1) * (T / N) ** 2 * alpha * N
    assert float(((e_out - e_in).abs() / e_in).max()) < 1e-5


def test_chunked_ragged_batch(oracle_mod):
    """A batch that spans more than one scratch chunk with a ragged tail."""
    N, alpha = 65536, 8          # 4 MiB of scratch per signal -> 32 signals per chunk
    batch = 35
    rng = np.random.default_rng(9)
    x = cplx(rng, (batch, N))
    X = gpu_alpha_dft(x, alpha, 1.0)
    for b in [0, 31, 32, 34]:
        bins = siggen.bin_subset(rng, alpha * N, 128)
        assert_close(X[b][bins], oracle_mod.alpha_dft_bins(x[b], alpha, 1.0, bins), "f32", f"sig {b}",
                     full_rms=spectrum_rms(x[b], 1.0))


PRECISION_FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                 "precision_2p22_a16_16384.npz")


def test_precision_form_2p22():
    """One complex64 signal, N = 2^22, alpha = 16 (2^26 bins), tones near
    Nyquist and at irrational multiples of 1/T: FP32 arithmetic with FP64
    twiddles.  The stated metric: relative L2 against the FP64 oracle on the
    seeded 16384-bin subset (oracle values precomputed by
    tests/golden/make_precision_fixture.py), bound 1e-5; the FP32-twiddle
    variant is measured beside it and must be worse."""
    import paper_2403_16665_amd as dd
    g = np.load(PRECISION_FIXTURE)
    N, alpha = int(g["N"]), int(g["alpha"])
    T = N * float(g["dt"])
    x = siggen.precision_tones(siggen.rngs(2, 1)[0], N)
    bins, ref = g["bins"], g["X"]
    X = gpu_alpha_dft(x[None, :], alpha, T)[0]
    r64 = rel_l2(X[bins], ref)
    assert r64 <= 1e-5, f"rel L2 on the 16384-bin subset {r64:.3e}"
    assert_close(X[bins], ref, "f32", "N=2^22 alpha=16", full_rms=spectrum_rms(x, T))
    X32 = gpu_alpha_dft(x[None, :], alpha, T, flags=dd.DD_TWIDDLE_FP32)[0]
    r32 = rel_l2(X32[bins], ref)
    print(f"precision N=2^22 alpha=16: rel L2 FP64 twiddles {r64:.3e}, FP32 twiddles {r32:.3e}")
    assert r32 > r64


def test_precision_form_2p22_every_schedule():
    """The same 2^22 x alpha 16 transform under every two-pass schedule the
    planner offers for it (the tuner, and so the timed benchmark, picks one of
    these), each against the oracle's 16384-bin fixture at the 1e-5 bound."""
    import torch
    import paper_2403_16665_amd as dd
    g = np.load(PRECISION_FIXTURE)
    N, alpha = int(g["N"]), int(g["alpha"])
    T = N * float(g["dt"])
    x = siggen.precision_tones(siggen.rngs(2, 1)[0], N)
    bins, ref = g["bins"], g["X"]
    xd = torch.from_numpy(x[None, :]).cuda()
    Xd = torch.empty((1, alpha * N), dtype=torch.complex64, device="cuda")
    idx = torch.from_numpy(bins).cuda()
    cands = dd.dense_dft_sched_candidates(N, alpha, 1, dd.DD_C64)
    assert cands, "no schedule for 2^22 x alpha 16"
    for sc in cands:
        plan = dd.dense_dft_plan_sched(N, alpha, T, 1, dd.DD_C64, sc)
        sc = sc.as_dict()
        Xd.zero_()
        dd.dense_dft_exec(plan, xd, Xd)
        got = Xd[0][idx].cpu().numpy()
        r = rel_l2(got, ref)
        print(f"schedule {sc}: rel L2 {r:.3e}")
        assert r <= 1e-5, f"schedule {sc}: rel L2 on the 16384-bin subset {r:.3e}"
        del plan


def test_tone_on_fine_bin_single_peak(oracle_mod):
    """A complex tone exactly on fine bin m0 gives the unique maximum T*A at m0
    and exact zeros at the other bins congruent to m0 mod alpha."""
    N, alpha, m0 = 4096, 8, 12345
    M = alpha * N
    n = np.arange(N)
    x = np.exp(2j * np.pi * ((m0 * n) % M) / M).astype(np.complex64)
    T = 4.096
    X = gpu_alpha_dft(x[None, :], alpha, T)[0]
    mags = np.abs(X)
    assert int(np.argmax(mags)) == m0
    assert abs(mags[m0] - T) < 1e-5 * T
    same = np.arange(m0 % alpha, M, alpha)
    same = same[same != m0]
    assert np.max(mags[same]) < 1e-5 * T


def test_fp32_twiddle_variant_is_worse_but_bounded(oracle_mod):
    """The FP32-twiddle variant (angle and sin/cos in FP32 from the exact
    integer exponent) still meets 1e-5 at moderate N, with larger error than
    the default FP64-generated twiddles."""
    import paper_2403_16665_amd as dd
    N, alpha = 1 << 16, 16
    x = cplx(np.random.default_rng(3), (1, N))
    bins = siggen.bin_subset(np.random.default_rng(4), alpha * N, 1024)
    ref = oracle_mod.alpha_dft_bins(x[0], alpha, 1.0, bins)
    e64 = rel_l2(gpu_alpha_dft(x, alpha, 1.0, flags=dd.DD_TWIDDLE_FP64)[0][bins], ref)
    e32 = rel_l2(gpu_alpha_dft(x, alpha, 1.0, flags=dd.DD_TWIDDLE_FP32)[0][bins], ref)
    assert e64 < 1e-6
    assert e32 < 1e-5
    assert e32 > e64


def test_max_size_sampled(oracle_mod):
    """alpha*N = 2^28 (N = 2^24 = 4096 x 4096, alpha = 16): 2 GiB of output."""
    N, alpha = 1 << 24, 16
    rng = np.random.default_rng(10)
    x = cplx(rng, (1, N))
    X = gpu_alpha_dft(x, alpha, 1.0)[0]
    bins = siggen.bin_subset(rng, alpha * N, 48)
    assert_close(X[bins], oracle_mod.alpha_dft_bins(x[0], alpha, 1.0, bins), "f32", "2^28 bins",
                 full_rms=spectrum_rms(x[0], 1.0))


def test_explicit_workspace_and_stream(oracle_mod):
    import torch
    import paper_2403_16665_amd as dd
    N, alpha, batch = 16384, 4, 3
    rng = np.random.default_rng(11)
    x = cplx(rng, (batch, N))
    plan = dd.dense_dft_plan(N, alpha, 1.0, batch, dd.DD_C64)
    ws_bytes = dd.dense_dft_workspace_size(plan)
    assert ws_bytes > 0
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    xd = torch.from_numpy(x).cuda()
    Xd = torch.empty((batch, alpha * N), dtype=torch.complex64, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    dd.dense_dft_exec(plan, xd, Xd, workspace=ws, stream=s.cuda_stream)
    s.synchronize()
    X = Xd.cpu().numpy()
    for b in range(batch):
        assert_close(X[b], oracle_mod.alpha_dft(x[b], alpha, 1.0), "f32", f"sig {b}")


def test_exec_rejects_bad_pointers():
    import torch
    import paper_2403_16665_amd as dd
    plan = dd.dense_dft_plan(1024, 4, 1.0, 2, dd.DD_C64)
    x = torch.zeros((2, 1024), dtype=torch.complex64, device="cuda")
    X = torch.zeros((2, 4096), dtype=torch.complex64, device="cuda")
    vp = dd._vp
    assert dd._lib.dense_dft_exec(plan.handle, None, vp(X.data_ptr()), None, None) == 1
    assert dd._lib.dense_dft_exec(plan.handle, vp(x.data_ptr()), None, None, None) == 1
    # misaligned output
    assert dd._lib.dense_dft_exec(plan.handle, vp(x.data_ptr()), vp(X.data_ptr() + 4), None, None) == 1
    # overlapping input and output
    big = torch.zeros(2 * 4096 + 2 * 1024, dtype=torch.complex64, device="cuda")
    assert dd._lib.dense_dft_exec(plan.handle, vp(big.data_ptr()), vp(big.data_ptr() + 8 * 1024),
                                  None, None) == 1
    torch.cuda.synchronize()


def test_unsupported_lengths():
    import paper_2403_16665_amd as dd
    for N in (7, 25, 9, 3 * 5 * 1024, 1 << 25):
        with pytest.raises(dd.DenseDFTError) as e:
            dd.dense_dft_plan(N, 2, 1.0, 1, dd.DD_C64)
        assert e.value.status == 2, N
