"""GPU tests at the largest transform the library accepts: alpha*N = 2^31
bins (16 GiB of complex64 output, and as much scratch), with N = N1*N2 at
the longest compiled pass lengths.  Checked on a seeded bin sample against
the FP64 oracle and, over the whole spectrum, by Parseval's relation
(eq. (8)): sum_m |X_m|^2 = (T/N)^2 alpha N sum_n |x_n|^2 for integer alpha."""
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


@pytest.mark.parametrize("N,alpha", [(1 << 24, 128), (3 << 22, 170)])
def test_largest_transform(oracle_mod, N, alpha):
    import torch
    import paper_2403_16665_amd as dd
    M = alpha * N
    assert M <= 1 << 31
    T = N * 1e-3
    x = siggen.tones_complex(np.random.default_rng(41), N, 1e-3)
    xd = torch.from_numpy(x).cuda()
    plan = dd.dense_dft_plan(N, alpha, T, 1, dd.DD_C64)
    sched = dd.dense_dft_plan_get_sched(plan)
    assert sched["passes"] == 2 and sched["N1"] * sched["N2"] == N
    X = torch.empty(M, dtype=torch.complex64, device="cuda")
    dd.dense_dft_exec(plan, xd, X)
    torch.cuda.synchronize()
    dd.dense_dft_destroy(plan)
    # bins near both ends, at multiples of alpha and at random
    rng = np.random.default_rng(5)
    bins = np.unique(np.concatenate([[0, 1, alpha - 1, alpha, M // 2, M - alpha, M - 1],
                                     siggen.bin_subset(rng, M, 9)]))
    got = X[torch.from_numpy(bins).cuda()].cpu().numpy()
    ref = oracle_mod.alpha_dft_bins(x, alpha, T, bins)
    assert_close(got, ref, "f32", f"N={N} alpha={alpha}", full_rms=spectrum_rms(x, T))
    # the whole spectrum's energy, accumulated in FP64 on the device
    energy = 0.0
    step = 1 << 27
    for i in range(0, M, step):
        energy += float(X[i:i + step].abs().double().pow(2).sum())
    expect = (T / N) ** 2 * M * float(np.sum(np.abs(x.astype(np.complex128)) ** 2))
    assert abs(energy - expect) <= 1e-5 * expect, (energy, expect)
    del X, xd
    torch.cuda.empty_cache()
