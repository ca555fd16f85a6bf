"""Seeded random sweep: (N, alpha, batch, input dtype, schedule) drawn over
the supported space -- powers of two and 3 * 2^a, 5 * 2^a lengths, alpha up
to 17, ragged batches, real and complex input in both precisions, the
planner's schedule or a random candidate -- each checked on seeded bins
against the oracle."""
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
