"""GPU parity of real-input transforms against the FP64 oracle.

For real samples the spectrum is Hermitian, X_{alpha N - m} = conj(X_m)
(Section 2: x real gives the negative-frequency half as conjugates).  The
two-pass schedule uses it: pass 1 stores only the scratch rows
m1 <= alpha N1 / 2 and pass 2 writes the other rows as conjugate mirrors.
Every two-pass schedule the planner offers is checked bin by bin, the
mirrored bins are checked to be exact conjugates, and the real path is
compared with the complex path on the same samples.
"""
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


def exact_mirror_bins(M, A):
    """Bins m whose mirror alpha N - m the kernel writes as the conjugate of
    the same stored value: rows 1 <= m1 < A - floor(A / 2) of A = alpha N1."""
    m = np.arange(M)
    m1 = m % A
    return m[(m1 >= 1) & (m1 < A - A // 2)]


def check_mirror(X, M, A, what):
    m = exact_mirror_bins(M, A)
    bad = np.flatnonzero(X[(M - m) % M] != np.conj(X[m]))
    assert bad.size == 0, f"{what}: {bad.size} mirrored bins differ from the conjugate, first m={m[bad[0]]}"


# (N, alpha): powers of two, 3 * 2^a and 5 * 2^a lengths, odd and even alpha N1
SHAPES = [(256, 16), (4096, 4), (8192, 2), (16384, 3), (48, 256), (3 * 2 ** 12, 5), (5 * 2 ** 11, 4),
          (5 * 2 ** 11, 3)]


@pytest.mark.parametrize("N,alpha", SHAPES)
@pytest.mark.parametrize("dtype,kind", [(np.float32, "f32"), (np.float64, "f64")])
def test_real_every_two_pass_schedule_every_bin(oracle_mod, N, alpha, dtype, kind):
    import torch
    import paper_2403_16665_amd as dd
    code = dd.DD_F32 if dtype == np.float32 else dd.DD_F64
    rng = np.random.default_rng(31 * N + alpha)
    batch = 3
    x = rng.standard_normal((batch, N)).astype(dtype)
    T = 1.5
    refs = [oracle_mod.alpha_dft(x[b], alpha, T) for b in range(batch)]
    xd = torch.from_numpy(x).cuda()
    M = alpha * N
    cands = [sc for sc in dd.dense_dft_sched_candidates(N, alpha, batch, code) if sc.passes == 2]
    assert cands, f"no two-pass schedule for N={N} alpha={alpha}"
    for sc in cands:
        plan = dd.dense_dft_plan_sched(N, alpha, T, batch, code, sc)
        passes, N1, _ = dd.dense_dft_plan_info(plan)
        assert passes == 2
        X = dd.alpha_dft(xd, alpha, T, plan=plan).cpu().numpy()
        for b in range(batch):
            what = f"real {dtype.__name__} N={N} alpha={alpha} schedule {sc.as_dict()} signal {b}"
            assert_close(X[b], refs[b], kind, what)
            check_mirror(X[b], M, alpha * N1, what)


SINGLE_N = [1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192,
            256, 320, 384, 512, 640, 768, 1024, 1280, 1536, 2048, 2560, 3072, 4096]


@pytest.mark.parametrize("N", SINGLE_N)
@pytest.mark.parametrize("dtype,kind", [(np.float32, "f32"), (np.float64, "f64")])
def test_real_one_pass_every_bin(oracle_mod, N, dtype, kind):
    """One-pass transforms of real signals transform only j <= alpha/2 and
    write the bins alpha (N - 1 - k) + alpha - j as conjugates of
    alpha k + j: every bin against the oracle, and those bins exact."""
    import torch
    import paper_2403_16665_amd as dd
    code = dd.DD_F32 if dtype == np.float32 else dd.DD_F64
    for alpha in (1, 2, 3, 5, 8, 16):
        rng = np.random.default_rng(17 * N + alpha)
        x = rng.standard_normal((3, N)).astype(dtype)
        T = 0.5
        try:  # the one-pass schedule (the planner runs spectra above 32 KiB in two passes)
            plan = dd.dense_dft_plan_sched(N, alpha, T, 3, code, dd.make_sched(passes=1, N1=N, N2=1))
        except dd.DenseDFTError:
            continue  # alpha N too large for one pass in this precision
        assert dd.dense_dft_plan_info(plan)[0] == 1
        X = dd.alpha_dft(torch.from_numpy(x).cuda(), alpha, T, plan=plan).cpu().numpy()
        M = alpha * N
        m = np.arange(M)
        j = m % alpha
        mirrored = m[(j >= 1) & (2 * j > alpha)]
        for b in range(3):
            what = f"real {dtype.__name__} one pass N={N} alpha={alpha} signal {b}"
            assert_close(X[b], oracle_mod.alpha_dft(x[b], alpha, T), kind, what)
            assert np.array_equal(X[b][mirrored], np.conj(X[b][M - mirrored])), what


def test_real_matches_complex_path_default_shape(oracle_mod):
    """256 x 65536 real float32 at alpha = 8 (the default workload's shape):
    the real path and the complex path on the same samples agree over the
    whole spectrum; sampled bins match the oracle."""
    import torch
    import paper_2403_16665_amd as dd
    N, alpha, batch, T = 65536, 8, 256, 65.536
    g = siggen.rngs(41, 1)[0]
    xr = torch.from_numpy(g.standard_normal((batch, N)).astype(np.float32)).cuda()
    plan = dd.dense_dft_plan(N, alpha, T, batch, dd.DD_F32)
    passes, N1, _ = dd.dense_dft_plan_info(plan)
    assert passes == 2
    Xr = dd.alpha_dft(xr, alpha, T, plan=plan)
    Xc = dd.alpha_dft(xr.to(torch.complex64), alpha, T)
    torch.cuda.synchronize()
    x_np = xr.cpu().numpy()
    rng = np.random.default_rng(2)
    for b in (0, 1, 31, 32, 255):
        got, ref = Xr[b].cpu().numpy(), Xc[b].cpu().numpy()
        assert_same(got, ref, f"real vs complex path, signal {b}")
        check_mirror(got, alpha * N, alpha * N1, f"signal {b}")
        bins = siggen.bin_subset(rng, alpha * N, 128)
        assert_close(got[bins], oracle_mod.alpha_dft_bins(x_np[b], alpha, T, bins), "f32", f"signal {b}",
                     full_rms=spectrum_rms(x_np[b], T))


def test_real_chunked_ragged_batch(oracle_mod):
    """A real batch over more than one scratch chunk with a ragged tail."""
    import paper_2403_16665_amd as dd
    from parity import gpu_alpha_dft
    N, alpha, batch = 65536, 8, 35
    rng = np.random.default_rng(10)
    x = np.stack([siggen.tones_real(g, N, 1e-3, alpha)[0] for g in siggen.rngs(43, batch)]).astype(np.float32)
    X = gpu_alpha_dft(x, alpha, 1.0)
    plan = dd.dense_dft_plan(N, alpha, 1.0, batch, dd.DD_F32)
    _, N1, _ = dd.dense_dft_plan_info(plan)
    for b in [0, 31, 32, 34]:
        bins = siggen.bin_subset(rng, alpha * N, 128)
        assert_close(X[b][bins], oracle_mod.alpha_dft_bins(x[b], alpha, 1.0, bins), "f32", f"sig {b}",
                     full_rms=spectrum_rms(x[b], 1.0))
        check_mirror(X[b], alpha * N, alpha * N1, f"sig {b}")
