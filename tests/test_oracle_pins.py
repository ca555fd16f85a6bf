"""Pins for the FP64 oracle: facts the paper and the mathematics fix.

Each check is independent of the oracle's own code: a textbook library
routine (numpy's FFT), a closed form, an invariant, a hand-worked example
(tests/golden), or a second algorithm (the paper's radix-2 recursion, eq. (13)).
The mutation test at the end plants known mistakes in the oracle and shows
that these pins catch every one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import siggen

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-12


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rand_c(rng, N):
    return rng.standard_normal(N) + 1j * rng.standard_normal(N)


# --- alpha = 1 reduces to the conventional DFT (eq. (5) scaled as eq. (2)) ---
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7, 8, 12, 16, 30, 64, 100])
def test_alpha1_is_conventional_dft(oracle_mod, N):
    rng = np.random.default_rng(N)
    x = rand_c(rng, N)
    T = 1.7
    X = oracle_mod.alpha_dft(x, 1, T)
    assert rel(X, np.fft.fft(x) * T / N) < TOL


# --- integer alpha equals zero padding to alpha*N (the claim of Section 2) ---
@pytest.mark.parametrize("N", [1, 2, 3, 5, 8, 17, 64, 96])
@pytest.mark.parametrize("alpha", [2, 3, 4, 8, 16])
def test_integer_alpha_is_zero_padded_dft(oracle_mod, N, alpha):
    rng = np.random.default_rng(1000 * N + alpha)
    x = rand_c(rng, N)
    T = 0.37 * N
    X = oracle_mod.alpha_dft(x, alpha, T)
    ref = np.fft.fft(np.concatenate([x, np.zeros((alpha - 1) * N)])) * T / N
    assert X.shape == (alpha * N,)
    assert rel(X, ref) < TOL


def test_every_alpha_th_bin_is_the_coarse_bin(oracle_mod):
    """m = alpha k lands on the conventional grid: X_{alpha k} = (T/N) FFT_N(x)_k."""
    rng = np.random.default_rng(7)
    N, alpha, T = 48, 5, 2.5
    x = rand_c(rng, N)
    X = oracle_mod.alpha_dft_bins(x, alpha, T, alpha * np.arange(N))
    assert rel(X, np.fft.fft(x) * T / N) < TOL


# --- hand-worked golden examples ---
def test_hand_worked_examples(oracle_mod):
    with open(os.path.join(HERE, "golden", "hand_examples.json")) as f:
        g = json.load(f)
    for ex in g["examples"]:
        x = np.array([complex(a, b) for a, b in ex["x"]])
        want = np.array([complex(a, b) for a, b in ex["X"]])
        got = oracle_mod.alpha_dft(x, ex["alpha"], ex["T"])
        assert np.max(np.abs(got - want)) < 1e-14, ex["name"]


# --- closed forms ---
@pytest.mark.parametrize("alpha", [1, 2, 5, 16])
def test_single_sample_leaf(oracle_mod, alpha):
    """N = 1: the recursion leaf, alpha identical outputs (T/N) x_0."""
    x = np.array([0.3 - 1.25j])
    T = 0.8
    X = oracle_mod.alpha_dft(x, alpha, T)
    assert np.max(np.abs(X - T * x[0])) < 1e-15


@pytest.mark.parametrize("N,alpha,m0", [(64, 4, 37), (100, 3, 1), (32, 8, 255), (60, 1, 7)])
def test_on_fine_bin_tone(oracle_mod, N, alpha, m0):
    """A complex tone exactly on fine bin m0: the peak is T*A*e^{i phi}, bins
    congruent to m0 mod alpha vanish, the rest follow the Dirichlet kernel
    (T/N) A e^{i phi} e^{-i pi d (N-1)/M} sin(pi d/alpha) / sin(pi d/M), d = m - m0."""
    M = alpha * N
    A, phi, T = 1.3, 0.7, 2.0
    n = np.arange(N)
    x = A * np.exp(1j * phi) * np.exp(2j * np.pi * ((m0 * n) % M) / M)
    X = oracle_mod.alpha_dft(x, alpha, T)
    m = np.arange(M)
    d = m - m0
    ref = np.empty(M, dtype=complex)
    ref[d == 0] = T * A * np.exp(1j * phi)
    on = (d % alpha == 0) & (d != 0)
    ref[on] = 0.0
    oth = d % alpha != 0
    dd = d[oth].astype(float)
    ref[oth] = (T / N) * A * np.exp(1j * phi) * np.exp(-1j * np.pi * dd * (N - 1) / M) \
        * np.sin(np.pi * dd / alpha) / np.sin(np.pi * dd / M)
    assert np.max(np.abs(X - ref)) < 1e-12 * T * A
    # the unique argmax is the tone's bin
    mags = np.abs(X)
    assert int(np.argmax(mags)) == m0
    assert np.sum(mags >= mags[m0] * (1 - 1e-12)) == 1


@pytest.mark.parametrize("N,alpha", [(1, 1), (7, 1), (16, 2), (30, 3), (64, 8), (5, 16)])
def test_parseval(oracle_mod, N, alpha):
    """Orthogonality eq. (8) gives sum|X|^2 = (T/N)^2 alpha N sum|x|^2 for integer alpha >= 1."""
    rng = np.random.default_rng(N * 31 + alpha)
    x = rand_c(rng, N)
    T = 1.9
    X = oracle_mod.alpha_dft(x, alpha, T)
    lhs = np.sum(np.abs(X) ** 2)
    rhs = (T / N) ** 2 * alpha * N * np.sum(np.abs(x) ** 2)
    assert abs(lhs - rhs) / rhs < 1e-12


@pytest.mark.parametrize("N,alpha", [(16, 4), (33, 3), (1024, 4)])
def test_hermitian_symmetry_for_real_input(oracle_mod, N, alpha):
    rng = np.random.default_rng(N + alpha)
    x = rng.standard_normal(N)
    X = oracle_mod.alpha_dft(x, alpha, 1.0)
    M = alpha * N
    mirror = X[(M - np.arange(M)) % M]
    assert np.max(np.abs(mirror - np.conj(X))) < 1e-12 * np.max(np.abs(X))


def test_linearity(oracle_mod):
    rng = np.random.default_rng(3)
    N, alpha, T = 40, 3, 0.9
    a, b = 0.7 - 0.2j, -1.1 + 0.4j
    x, y = rand_c(rng, N), rand_c(rng, N)
    lhs = oracle_mod.alpha_dft(a * x + b * y, alpha, T)
    rhs = a * oracle_mod.alpha_dft(x, alpha, T) + b * oracle_mod.alpha_dft(y, alpha, T)
    assert rel(lhs, rhs) < TOL


# --- second algorithm: the paper's radix-2 recursion, eq. (10)-(13) ---
def eq13_recursion(x, alpha):
    """Unscaled alpha-DFT by the even/odd split of Section 3: Y, Z are the
    half-length alpha-DFTs of the even and odd samples (alpha N/2 outputs each),
    X_l = Y_l + W_{alpha N}^l Z_l and X_{l + alpha N/2} = Y_l - W^l Z_l.  The
    recursion stops at one sample, whose alpha outputs all equal it."""
    N = len(x)
    if N == 1:
        return [x[0]] * alpha
    Y = eq13_recursion(x[0::2], alpha)
    Z = eq13_recursion(x[1::2], alpha)
    M = alpha * N
    h = M // 2
    out = [0j] * M
    for l in range(h):
        w = complex(math.cos(2 * math.pi * l / M), -math.sin(2 * math.pi * l / M))
        out[l] = Y[l] + w * Z[l]
        out[l + h] = Y[l] - w * Z[l]
    return out


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("alpha", [1, 2, 3, 4, 8])
def test_matches_eq13_radix2_recursion(oracle_mod, N, alpha):
    rng = np.random.default_rng(N * 7 + alpha)
    x = rand_c(rng, N)
    T = 3.1
    ref = np.array(eq13_recursion(list(x), alpha)) * T / N
    assert rel(oracle_mod.alpha_dft(x, alpha, T), ref) < TOL


# --- inverse, eq. (7) second line with eq. (8) ---
@pytest.mark.parametrize("N,alpha", [(8, 1), (12, 2), (25, 4)])
def test_inverse_round_trip(oracle_mod, N, alpha):
    """x_n = (1/(alpha N)) sum_m e^{+2 pi i mn/(alpha N)} X'_m with X' = (N/T) X;
    by eq. (8) the same sum vanishes for N <= n < alpha N."""
    rng = np.random.default_rng(N + 100 * alpha)
    x = rand_c(rng, N)
    T = 0.6
    X = oracle_mod.alpha_dft(x, alpha, T)
    back = np.fft.ifft(X * N / T)
    assert np.max(np.abs(back[:N] - x)) < 1e-12
    if alpha > 1:
        assert np.max(np.abs(back[N:])) < 1e-12


# --- subset evaluation, input promotion, arguments, large-M path ---
def test_subset_equals_full(oracle_mod):
    rng = np.random.default_rng(11)
    N, alpha = 96, 3
    x = rand_c(rng, N)
    full = oracle_mod.alpha_dft(x, alpha, 1.0)
    bins = siggen.bin_subset(rng, alpha * N, 50)
    assert np.array_equal(oracle_mod.alpha_dft_bins(x, alpha, 1.0, bins), full[bins])


def test_float32_input_promoted_exactly(oracle_mod):
    rng = np.random.default_rng(12)
    x32 = (rand_c(rng, 64)).astype(np.complex64)
    a = oracle_mod.alpha_dft(x32, 2, 1.0)
    b = oracle_mod.alpha_dft(x32.astype(np.complex128), 2, 1.0)
    assert np.array_equal(a, b)


def test_rejects_bad_arguments(oracle_mod):
    x = np.ones(4)
    with pytest.raises(ValueError):
        oracle_mod.alpha_dft_bins(x, 2, 1.0, [8])
    with pytest.raises(ValueError):
        oracle_mod.alpha_dft_bins(x, 0, 1.0, [0])
    with pytest.raises(ValueError):
        oracle_mod.alpha_dft_bins(x, 2, 1.0, [-1])


def test_large_M_direct_sincos_path(oracle_mod):
    """alpha N above the oracle's table limit (2^22) takes the direct libm path."""
    rng = np.random.default_rng(13)
    N, alpha = 1 << 17, 64          # M = 2^23
    x = rand_c(rng, N)
    bins = siggen.bin_subset(rng, alpha * N, 24)
    got = oracle_mod.alpha_dft_bins(x, alpha, 1.0, bins)
    ref = np.fft.fft(np.concatenate([x, np.zeros((alpha - 1) * N)]))[bins] / N
    assert rel(got, ref) < 1e-11


# --- the oracle's own rounding, against extended precision ---
def longdouble_bins(x, alpha, T, bins):
    """The definition summed in x86 80-bit long double: exponents reduced
    exactly in integers, cos/sin of the long-double angle."""
    N = len(x)
    M = alpha * N
    ld = np.longdouble
    xr = np.asarray(x.real, dtype=ld)
    xi = np.asarray(x.imag, dtype=ld)
    n = np.arange(N, dtype=np.int64)
    two_pi = ld(2) * np.arccos(ld(-1))
    out = []
    for m in bins:
        q = (int(m) * n) % M
        th = two_pi * q.astype(ld) / ld(M)
        c, s = np.cos(th), np.sin(th)
        re = np.sum(xr * c + xi * s)
        im = np.sum(xi * c - xr * s)
        out.append(complex(float(re * ld(T) / ld(N)), float(im * ld(T) / ld(N))))
    return np.array(out)


@pytest.mark.skipif(np.finfo(np.longdouble).eps > 1e-18, reason="long double is not 80-bit here")
@pytest.mark.parametrize("N,alpha", [(4096, 8), (4096, 1 << 14)])
def test_oracle_rounding_against_long_double(oracle_mod, N, alpha):
    """Random bins of a random signal, at a small M and at M = 2^26 (the
    large-M twiddle path): the FP64 oracle is within 1e-13 of the sum in
    extended precision."""
    rng = np.random.default_rng(21)
    x = rand_c(rng, N)
    bins = siggen.bin_subset(rng, alpha * N, 64)
    got = oracle_mod.alpha_dft_bins(x, alpha, 0.75, bins)
    ref = longdouble_bins(x, alpha, 0.75, bins)
    assert rel(got, ref) < 1e-13


# --- planted mistakes must be caught ---
def _pins_pass(oracle_mod, mutation):
    rng = np.random.default_rng(99)
    ok = True
    x = rand_c(rng, 16)
    T = 1.7
    ok &= rel(oracle_mod.alpha_dft(x, 1, T, mutation=mutation), np.fft.fft(x) * T / 16) < TOL
    x = rand_c(rng, 8)
    ref = np.fft.fft(np.concatenate([x, np.zeros(16)])) * T / 8
    got = oracle_mod.alpha_dft(x, 3, T, mutation=mutation)
    ok &= got.shape == ref.shape and rel(got, ref) < TOL
    with open(os.path.join(HERE, "golden", "hand_examples.json")) as f:
        for ex in json.load(f)["examples"]:
            xx = np.array([complex(a, b) for a, b in ex["x"]])
            want = np.array([complex(a, b) for a, b in ex["X"]])
            got = oracle_mod.alpha_dft(xx, ex["alpha"], ex["T"], mutation=mutation)
            ok &= bool(np.max(np.abs(got - want)) < 1e-14)
    return bool(ok)


def test_pins_accept_the_oracle(oracle_mod):
    assert _pins_pass(oracle_mod, 0)


@pytest.mark.parametrize("mutation", [1, 2, 3, 4, 5, 6])
def test_pins_catch_planted_mistakes(oracle_mod, mutation):
    """1 sign of exponent, 2 dropped last term, 3 off-by-one sample index,
    4 scale 1/N instead of T/N, 5 alpha ignored, 6 real/imag swapped."""
    assert not _pins_pass(oracle_mod, mutation)


# --- the seeded generators are deterministic ---
def test_generators_deterministic():
    a = siggen.tones_complex(siggen.rngs(1, 2)[1], 256, 1e-3)
    b = siggen.tones_complex(siggen.rngs(1, 2)[1], 256, 1e-3)
    assert np.array_equal(a, b)
    x1, p1 = siggen.tones_real(siggen.rngs(0, 1)[0], 1024, 1e-3, 4)
    x2, p2 = siggen.tones_real(siggen.rngs(0, 1)[0], 1024, 1e-3, 4)
    assert np.array_equal(x1, x2)
    fr = (p1[0] * 4 * 1.024) % 1.0
    assert np.all((fr >= 0.1) & (fr <= 0.9))
    mix = siggen.uneven_mix(siggen.rngs(3, 1)[0], 1000)
    assert len(mix) == 1000
    assert all(n in siggen.uneven_sizes() and a in siggen.UNEVEN_ALPHAS for n, a in mix)


# --- the oracle's inverse transform (eq. (7) second line, 1/(alpha T)) ---
@pytest.mark.parametrize("N,alpha", [(16, 1), (12, 3), (25, 4), (40, 8)])
def test_inverse_against_library_ifft(oracle_mod, N, alpha):
    """x_n = (1/(alpha T)) sum_m X_m e^{+2 pi i mn/(alpha N)} = (N/T) ifft(X)_n
    for any spectrum X, not only forward spectra (numpy's ifft carries 1/(alpha N))."""
    rng = np.random.default_rng(7 * N + alpha)
    X = rand_c(rng, alpha * N)
    T = 1.7
    got = oracle_mod.inverse_alpha_dft_samples(X, alpha, T, np.arange(alpha * N))
    ref = np.fft.ifft(X) * (N / T)
    assert rel(got, ref) < TOL


@pytest.mark.parametrize("N,alpha", [(8, 1), (24, 2), (20, 5), (64, 16)])
def test_inverse_round_trip_and_vanishing_tail(oracle_mod, N, alpha):
    """The inverse undoes the forward transform on the N samples, and the
    samples N <= n < alpha N of the same sum vanish (the padded zeros)."""
    rng = np.random.default_rng(N + alpha)
    x = rand_c(rng, N)
    T = 0.9
    X = oracle_mod.alpha_dft(x, alpha, T)
    assert rel(oracle_mod.inverse_alpha_dft(X, alpha, T), x) < TOL
    if alpha > 1:
        tail = oracle_mod.inverse_alpha_dft_samples(X, alpha, T, np.arange(N, alpha * N))
        assert np.max(np.abs(tail)) < 1e-12 * np.max(np.abs(x))


def test_inverse_single_bin_closed_form(oracle_mod):
    """X = delta at m0: x_n = e^{2 pi i m0 n/(alpha N)} / (alpha T)."""
    N, alpha, T, m0 = 30, 4, 2.5, 37
    X = np.zeros(alpha * N, dtype=np.complex128)
    X[m0] = 1.0
    n = np.arange(N)
    ref = np.exp(2j * np.pi * m0 * n / (alpha * N)) / (alpha * T)
    assert rel(oracle_mod.inverse_alpha_dft(X, alpha, T), ref) < TOL


def test_inverse_large_M_direct_sincos_path(oracle_mod):
    """alpha N above the oracle's table limit (2^22): the inverse takes the
    direct libm path.  The spectrum is numpy's FFT of the zero-padded signal
    (the forward transform, Section 4's zero-padding identity), so the
    inverse must return x_n for n < N and zero for N <= n < alpha N; each
    sampled value is also (N/T) ifft(X)_n of the same spectrum."""
    rng = np.random.default_rng(17)
    N, alpha, T = 1 << 17, 64, 3.0     # M = 2^23
    x = rand_c(rng, N)
    X = np.fft.fft(np.concatenate([x, np.zeros((alpha - 1) * N)])) * (T / N)
    n_lo = np.sort(rng.choice(N, 12, replace=False))
    n_hi = N + np.sort(rng.choice((alpha - 1) * N, 12, replace=False))
    got = oracle_mod.inverse_alpha_dft_samples(X, alpha, T, np.concatenate([n_lo, n_hi]))
    assert rel(got[:12], x[n_lo]) < 1e-11
    assert np.max(np.abs(got[12:])) < 1e-11 * np.max(np.abs(x[n_lo]))
    ref = np.fft.ifft(X) * (N / T)
    assert rel(got, ref[np.concatenate([n_lo, n_hi])]) < 1e-10


@pytest.mark.parametrize("mutation", [1, 2, 3, 4])
def test_inverse_pins_reject_planted_mistakes(oracle_mod, mutation):
    """Each planted mistake of the inverse fails at least one of the pins above."""
    rng = np.random.default_rng(99)
    N, alpha, T = 24, 3, 1.3
    X = rand_c(rng, alpha * N)
    x = rand_c(rng, N)
    fails = []
    got = oracle_mod.inverse_alpha_dft_samples(X, alpha, T, np.arange(alpha * N), mutation=mutation)
    fails.append(rel(got, np.fft.ifft(X) * (N / T)) >= TOL)
    Xf = oracle_mod.alpha_dft(x, alpha, T)
    fails.append(rel(oracle_mod.inverse_alpha_dft(Xf, alpha, T, mutation=mutation), x) >= TOL)
    assert any(fails)


# --- alpha = 1/p (Section 2, alpha < 1) ---
@pytest.mark.parametrize("N,p", [(12, 1), (12, 3), (40, 4), (60, 5), (64, 16)])
def test_decimated_against_library_fft(oracle_mod, N, p):
    """X_m = (T/N) sum_n x_n e^{-2 pi i mn/(N/p)} is the textbook DFT at every
    p-th bin, and also the DFT of length N/p of the folded sequence
    x'_r = sum_k x_{r + k N/p} (the periodicity the paper's alpha < 1 case uses)."""
    rng = np.random.default_rng(N * p)
    x = rand_c(rng, N)
    T = 2.2
    got = oracle_mod.decimated_dft(x, p, T)
    assert rel(got, np.fft.fft(x)[::p] * T / N) < TOL
    folded = x.reshape(p, N // p).sum(axis=0)
    assert rel(got, np.fft.fft(folded) * T / N) < TOL


def test_decimated_rejects_non_divisor(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.decimated_dft(np.ones(10), 3, 1.0)
