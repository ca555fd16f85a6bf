"""The zero-padding identity the paper starts from (Section 2): for integer
alpha the alpha-dense DFT equals the DFT of the sequence padded with
(alpha-1) N zeros.  On the GPU: the alpha-dense plan against this library's
own alpha = 1 plan at length alpha*N on the padded input (the ablation the
benchmark times), whole spectra compared, both also against the oracle."""
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


@pytest.mark.parametrize("N,alpha,batch", [(4096, 8, 3), (65536, 8, 2), (3 * 2 ** 12, 4, 2), (5 * 2 ** 10, 2, 2), (1024, 3, 4)])
def test_alpha_dense_equals_padded_fft(oracle_mod, N, alpha, batch):
    import torch
    import paper_2403_16665_amd as dd
    T = N * 1e-3
    M = alpha * N
    x = np.stack([siggen.tones_complex(g, N, 1e-3) for g in siggen.rngs(9, batch)])
    xd = torch.from_numpy(x).cuda()
    xp = torch.zeros(batch, M, dtype=torch.complex64, device="cuda")
    xp[:, :N] = xd
    X = dd.alpha_dft(xd, alpha, T)
    Xp = dd.alpha_dft(xp, 1, alpha * T)   # T/N = (alpha T) / (alpha N)
    torch.cuda.synchronize()
    X, Xp = X.cpu().numpy(), Xp.cpu().numpy()
    rng = np.random.default_rng(2)
    for b in range(batch):
        assert_same(Xp[b], X[b], f"padded vs alpha-dense, signal {b}")
        bins = siggen.bin_subset(rng, M, 128)
        ref = oracle_mod.alpha_dft_bins(x[b], alpha, T, bins)
        assert_close(Xp[b][bins], ref, "f32", "padded FFT vs oracle", full_rms=spectrum_rms(x[b], T))
