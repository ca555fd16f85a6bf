"""GPU tests of the inverse alpha-transform (the reading of eq. (7), second
line, with the factor 1/(alpha T)): parity with the FP64 oracle's inverse on
arbitrary spectra, for one-pass and two-pass plans of both precisions, and
the round trip forward -> inverse back to the signal."""
import numpy as np
import pytest

import siggen
from parity import assert_close, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def spectra(rng, batch, M, dtype):
    X = (rng.standard_normal((batch, M)) + 1j * rng.standard_normal((batch, M)))
    return X.astype(dtype)


ONE_PASS = [(1, 4, 3), (16, 2, 5), (256, 8, 4), (1024, 4, 2), (3072, 3, 2), (320, 16, 3)]


@pytest.mark.parametrize("N,alpha,batch", ONE_PASS + [
    (8192, 4, 2), (65536, 8, 2), (3 * 2 ** 13, 5, 2), (5 * 2 ** 11, 2, 3), (4096, 16, 2)])
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_inverse_matches_oracle(oracle_mod, N, alpha, batch, dtype):
    import torch
    import paper_2403_16665_amd as dd
    rng = np.random.default_rng(N * 7 + alpha)
    M = alpha * N
    T = 0.37 * N
    X = spectra(rng, batch, M, dtype)
    code = dd.DD_C64 if dtype == np.complex64 else dd.DD_C128
    plan = None
    if (N, alpha, batch) in ONE_PASS:
        # the one-pass schedule wherever it fits (the planner runs spectra
        # above 32 KiB in two passes)
        try:
            plan = dd.dense_dft_plan_sched(N, alpha, T, batch, code, dd.make_sched(passes=1, N1=N, N2=1))
        except dd.DenseDFTError:
            plan = None
    x = dd.alpha_idft(torch.from_numpy(X).cuda(), alpha, T, plan=plan).cpu().numpy()
    kind = "f32" if dtype == np.complex64 else "f64"
    samples = np.arange(N) if N <= 4096 else siggen.bin_subset(rng, N, 512)
    for b in range(batch):
        ref = oracle_mod.inverse_alpha_dft_samples(X[b], alpha, T, samples)
        if len(samples) == N:
            assert_close(x[b], ref, kind, f"inverse N={N} alpha={alpha}")
        else:
            # for a white spectrum the output's energy spreads evenly over the
            # samples, so the sample RMS estimates the whole output's RMS
            assert_close(x[b][samples], ref, kind, f"inverse N={N} alpha={alpha}",
                         full_rms=np.sqrt(np.mean(np.abs(ref) ** 2)))


@pytest.mark.parametrize("N,alpha,batch,dtype", [
    (1024, 4, 3, np.complex64), (65536, 8, 4, np.complex64), (3 * 2 ** 12, 3, 2, np.complex64),
    (4096, 2, 2, np.float32), (2048, 16, 2, np.complex128), (1024, 1, 2, np.float64)])
def test_round_trip(N, alpha, batch, dtype):
    import torch
    import paper_2403_16665_amd as dd
    rng = np.random.default_rng(N + alpha)
    if np.issubdtype(dtype, np.complexfloating):
        x = np.stack([siggen.tones_complex(g, N, 1e-3) for g in siggen.rngs(12, batch)]).astype(dtype)
    else:
        x = rng.standard_normal((batch, N)).astype(dtype)
    T = N * 1e-3
    xd = torch.from_numpy(x).cuda()
    code = dd.dtype_code(xd.dtype)
    plan = dd.dense_dft_plan(N, alpha, T, batch, code)
    X = dd.alpha_dft(xd, alpha, T, plan=plan)
    back = torch.empty((batch, N), dtype=X.dtype, device="cuda")
    dd.dense_dft_exec_inverse(plan, X, back)
    torch.cuda.synchronize()
    back = back.cpu().numpy()
    tol = 1e-5 if X.dtype == torch.complex64 else 1e-12
    for b in range(batch):
        r = rel_l2(back[b], x[b].astype(back.dtype))
        assert r <= tol, f"round trip N={N} alpha={alpha} signal {b}: rel L2 {r:.3e}"
