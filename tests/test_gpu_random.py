"""Seeded random sweep: (N, alpha, batch, input dtype, schedule) drawn over
the supported space -- powers of two and 3 * 2^a, 5 * 2^a lengths, alpha up
to 17, ragged batches (up to 40 signals in the wide draws), real and complex
input in both precisions, the planner's schedule or a random candidate --
each checked on seeded bins against the oracle (the wide draws also invert
complex spectra back to their signals)."""
import numpy as np
import pytest

import siggen
from parity import assert_close, spectrum_rms

pytestmark = pytest.mark.gpu

LENGTHS = sorted({b << a for b in (1, 3, 5) for a in range(0, 19) if (b << a) <= (1 << 18)})


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def draw(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.choice(LENGTHS))
    alpha = int(rng.integers(1, 18))
    while alpha * N > (1 << 24):
        alpha = max(1, alpha // 2)
    return rng, N, alpha, int(rng.integers(1, 6)), int(rng.integers(0, 4)), bool(rng.integers(0, 2))


@pytest.mark.parametrize("seed", range(120))
def test_random_configuration(oracle_mod, seed):
    import torch
    import paper_2403_16665_amd as dd
    rng, N, alpha, batch, code, random_sched = draw(seed)
    dt = {dd.DD_F32: np.float32, dd.DD_C64: np.complex64, dd.DD_F64: np.float64, dd.DD_C128: np.complex128}[code]
    if np.issubdtype(dt, np.complexfloating):
        x = (rng.standard_normal((batch, N)) + 1j * rng.standard_normal((batch, N))).astype(dt)
    else:
        x = rng.standard_normal((batch, N)).astype(dt)
    T = float(rng.uniform(0.1, 10.0))
    if random_sched:
        cands = dd.dense_dft_sched_candidates(N, alpha, batch, code)
        sc = cands[int(rng.integers(0, len(cands)))]
        plan = dd.dense_dft_plan_sched(N, alpha, T, batch, code, sc)
    else:
        plan = dd.dense_dft_plan(N, alpha, T, batch, code)
    what = (f"seed {seed}: N={N} alpha={alpha} batch={batch} dtype={code} "
            f"schedule {dd.dense_dft_plan_get_sched(plan)}")
    X = dd.alpha_dft(torch.from_numpy(x).cuda(), alpha, T, plan=plan).cpu().numpy()
    kind = "f64" if code in (dd.DD_F64, dd.DD_C128) else "f32"
    M = alpha * N
    for b in range(batch):
        bins = siggen.bin_subset(rng, M, 96)
        full = None if len(bins) == M else spectrum_rms(x[b], T)
        assert_close(X[b][bins], oracle_mod.alpha_dft_bins(x[b], alpha, T, bins), kind, f"{what} signal {b}",
                     full_rms=full)


def draw_wide(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.choice(LENGTHS))
    alpha = int(rng.integers(1, 18))
    while alpha * N > (1 << 22):
        alpha = max(1, alpha // 2)
    return rng, N, alpha, int(rng.integers(1, 41)), int(rng.integers(0, 4)), bool(rng.integers(0, 3) > 0)


@pytest.mark.parametrize("seed", range(5000, 5200))
def test_random_wide_batches_and_round_trip(oracle_mod, seed):
    """As test_random_configuration with up to 40 signals (ragged last
    blocks of multi-signal one-pass shapes) and, for complex input, the
    inverse of the plan's own output back to the signal."""
    import torch
    import paper_2403_16665_amd as dd
    rng, N, alpha, batch, code, random_sched = draw_wide(seed)
    dt = {dd.DD_F32: np.float32, dd.DD_C64: np.complex64, dd.DD_F64: np.float64, dd.DD_C128: np.complex128}[code]
    if np.issubdtype(dt, np.complexfloating):
        x = (rng.standard_normal((batch, N)) + 1j * rng.standard_normal((batch, N))).astype(dt)
    else:
        x = rng.standard_normal((batch, N)).astype(dt)
    T = float(rng.uniform(0.1, 10.0))
    if random_sched:
        cands = dd.dense_dft_sched_candidates(N, alpha, batch, code)
        sc = cands[int(rng.integers(0, len(cands)))]
        plan = dd.dense_dft_plan_sched(N, alpha, T, batch, code, sc)
    else:
        plan = dd.dense_dft_plan(N, alpha, T, batch, code)
    what = (f"seed {seed}: N={N} alpha={alpha} batch={batch} dtype={code} "
            f"schedule {dd.dense_dft_plan_get_sched(plan)}")
    Xd = dd.alpha_dft(torch.from_numpy(x).cuda(), alpha, T, plan=plan)
    X = Xd.cpu().numpy()
    kind = "f64" if code in (dd.DD_F64, dd.DD_C128) else "f32"
    M = alpha * N
    for b in range(batch):
        bins = siggen.bin_subset(rng, M, 96)
        full = None if len(bins) == M else spectrum_rms(x[b], T)
        assert_close(X[b][bins], oracle_mod.alpha_dft_bins(x[b], alpha, T, bins), kind, f"{what} signal {b}",
                     full_rms=full)
    if np.issubdtype(dt, np.complexfloating):
        back = torch.empty((batch, N), dtype=Xd.dtype, device="cuda")
        dd.dense_dft_exec_inverse(plan, Xd, back)
        torch.cuda.synchronize()
        bk = back.cpu().numpy()
        for b in range(batch):
            r = np.linalg.norm(bk[b] - x[b]) / np.linalg.norm(x[b])
            assert r <= (1e-5 if code == dd.DD_C64 else 1e-12), f"{what} signal {b}: inverse round trip {r:.3e}"


@pytest.mark.parametrize("seed", range(20))
def test_random_batch_mix(oracle_mod, seed):
    """One persistent batch of 12 random items (lengths the batch kernel is
    built for and others, real float32 and complex64, alpha up to 17):
    sampled bins of every item against the oracle."""
    import torch
    import paper_2403_16665_amd as dd
    rng = np.random.default_rng(1000 + seed)
    small = [n for n in LENGTHS if 16 <= n <= (1 << 16)]
    items, xs, Xs = [], [], []
    for _ in range(12):
        N = int(rng.choice(small))
        alpha = int(rng.integers(1, 18))
        real = bool(rng.integers(0, 2))
        x = rng.standard_normal(N).astype(np.float32) if real else \
            (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
        xs.append(torch.from_numpy(x).cuda())
        Xs.append(torch.zeros(alpha * N, dtype=torch.complex64, device="cuda"))
        items.append((N, alpha, N * 1e-3, dd.DD_F32 if real else dd.DD_C64, x))
    torch.cuda.synchronize()
    dd.dense_dft_exec_many([(N, a, T, c, xs[i], Xs[i]) for i, (N, a, T, c, _) in enumerate(items)])
    for i, (N, a, T, c, x) in enumerate(items):
        bins = siggen.bin_subset(rng, a * N, 96)
        full = None if len(bins) == a * N else spectrum_rms(x, T)
        assert_close(Xs[i].cpu().numpy()[bins], oracle_mod.alpha_dft_bins(x, a, T, bins), "f32",
                     f"seed {seed} item {i}: N={N} alpha={a} dtype={c}", full_rms=full)


@pytest.mark.parametrize("seed", range(40))
def test_random_batch_mix_wide(oracle_mod, seed):
    """One persistent batch of 1 to 60 random items up to 2^18 samples and
    2^21 bins (real float32 and complex64, alpha up to 17): sampled bins of
    every item against the oracle."""
    import torch
    import paper_2403_16665_amd as dd
    rng = np.random.default_rng(7000 + seed)
    lengths = [n for n in LENGTHS if 16 <= n <= (1 << 18)]
    items, xs, Xs = [], [], []
    for _ in range(int(rng.integers(1, 61))):
        N = int(rng.choice(lengths))
        alpha = int(rng.integers(1, 18))
        while alpha * N > (1 << 21):
            alpha = max(1, alpha // 2)
        real = bool(rng.integers(0, 2))
        x = rng.standard_normal(N).astype(np.float32) if real else \
            (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
        xs.append(torch.from_numpy(x).cuda())
        Xs.append(torch.zeros(alpha * N, dtype=torch.complex64, device="cuda"))
        items.append((N, alpha, N * 1e-3, dd.DD_F32 if real else dd.DD_C64, x))
    torch.cuda.synchronize()
    dd.dense_dft_exec_many([(N, a, T, c, xs[i], Xs[i]) for i, (N, a, T, c, _) in enumerate(items)])
    for i, (N, a, T, c, x) in enumerate(items):
        bins = siggen.bin_subset(rng, a * N, 64)
        full = None if len(bins) == a * N else spectrum_rms(x, T)
        assert_close(Xs[i].cpu().numpy()[bins], oracle_mod.alpha_dft_bins(x, a, T, bins), "f32",
                     f"seed {seed} item {i}/{len(items)}: N={N} alpha={a} dtype={c}", full_rms=full)


@pytest.mark.parametrize("seed", range(20))
def test_random_inverse(oracle_mod, seed):
    """Inverse transforms of random spectra in both precisions, with the
    planner's schedule or a random candidate: sampled outputs against the
    oracle's inverse."""
    import torch
    import paper_2403_16665_amd as dd
    rng, N, alpha, batch, code, random_sched = draw(2000 + seed)
    cplx = np.complex128 if code in (dd.DD_F64, dd.DD_C128) else np.complex64
    code = dd.DD_C128 if cplx == np.complex128 else dd.DD_C64
    M = alpha * N
    X = (rng.standard_normal((batch, M)) + 1j * rng.standard_normal((batch, M))).astype(cplx)
    T = float(rng.uniform(0.1, 10.0))
    if random_sched:
        cands = dd.dense_dft_sched_candidates(N, alpha, batch, code)
        plan = dd.dense_dft_plan_sched(N, alpha, T, batch, code, cands[int(rng.integers(0, len(cands)))])
    else:
        plan = dd.dense_dft_plan(N, alpha, T, batch, code)
    x = plan.exec_inverse(torch.from_numpy(X).cuda()).cpu().numpy()
    kind = "f64" if code == dd.DD_C128 else "f32"
    for b in range(batch):
        samples = siggen.bin_subset(rng, N, 96)
        ref = oracle_mod.inverse_alpha_dft_samples(X[b], alpha, T, samples)
        full = None if len(samples) == N else np.sqrt(np.mean(np.abs(ref) ** 2))
        assert_close(x[b][samples], ref, kind, f"seed {seed}: inverse N={N} alpha={alpha} batch={batch}",
                     full_rms=full)
