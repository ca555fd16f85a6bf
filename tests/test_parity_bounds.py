"""CPU checks of the comparison rule the GPU parity tests use: a textbook
single-precision FFT of a strongly tonal signal passes it (so the bound is
not tighter than FP32 rounding), and the mistakes it exists to catch fail it:
a bin off by one, a wrong scale, one wrong twiddle, a conjugated spectrum."""
import numpy as np
import pytest

import siggen
from parity import assert_close, spectrum_rms


def tonal(N, seed=0):
    return siggen.tones_complex(np.random.default_rng(seed), N, 1e-3, sigma=0.01)


@pytest.mark.parametrize("N,alpha", [(4096, 4), (1 << 16, 8), (1 << 18, 2)])
def test_fp32_fft_passes(N, alpha):
    x = tonal(N)
    T = N * 1e-3
    ref = np.fft.fft(np.concatenate([x.astype(np.complex128), np.zeros((alpha - 1) * N)])) * (T / N)
    # numpy's FFT (single precision for complex64 input) on the same samples
    xp = np.concatenate([x, np.zeros((alpha - 1) * N, np.complex64)])
    got = np.fft.fft(xp).astype(np.complex64) * np.float32(T / N)
    got32 = got
    assert_close(got32, ref, "f32", "numpy single-precision FFT")
    rng = np.random.default_rng(1)
    bins = siggen.bin_subset(rng, alpha * N, 4096)
    assert_close(got32[bins], ref[bins], "f32", "sampled", full_rms=spectrum_rms(x, T))


def planted(N=1 << 14, alpha=4):
    x = tonal(N, 2)
    T = N * 1e-3
    ref = np.fft.fft(np.concatenate([x.astype(np.complex128), np.zeros((alpha - 1) * N)])) * (T / N)
    return x, T, ref


def test_bin_off_by_one_fails():
    x, T, ref = planted()
    with pytest.raises(AssertionError):
        assert_close(np.roll(ref, 1), ref, "f32")


def test_wrong_scale_fails():
    x, T, ref = planted()
    with pytest.raises(AssertionError):
        assert_close(ref * (1 + 1e-4), ref, "f32")


def test_one_wrong_twiddle_fails():
    """One twiddle of the last radix-2 stage taken at a wrong index (a quarter
    turn away): an error of the order of the value it multiplies, in two bins
    only.  (A twiddle off by a single step of 2 pi / M changes a bin by about
    1e-4 of one term, the size of FP32 rounding: not what this rule is for.)"""
    x, T, ref = planted()
    M = ref.size
    half = M // 2
    even = np.fft.fft(np.concatenate([x, np.zeros(M - x.size)])[0::2].astype(np.complex128))
    odd = np.fft.fft(np.concatenate([x, np.zeros(M - x.size)])[1::2].astype(np.complex128))
    tw = np.exp(-2j * np.pi * np.arange(half) / M)
    tw[7] = np.exp(-2j * np.pi * (7 + M // 4) / M)
    bad = np.concatenate([even + tw * odd, even - tw * odd]) * (T / x.size)
    with pytest.raises(AssertionError):
        assert_close(bad, ref, "f32")
    rng = np.random.default_rng(5)
    bins = np.union1d(siggen.bin_subset(rng, M, 512), [7, 7 + half])
    with pytest.raises(AssertionError):
        assert_close(bad[bins], ref[bins], "f32", full_rms=spectrum_rms(x, T))


def test_conjugated_spectrum_fails():
    x, T, ref = planted()
    with pytest.raises(AssertionError):
        assert_close(np.conj(ref), ref, "f32")
