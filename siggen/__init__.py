"""Seeded synthetic workloads for the alpha-dense DFT (tests, benchmark, oracle checks).

This module only draws random numbers and synthesises tone-plus-noise
signals; it holds none of the transform's arithmetic.  Both the GPU path's
tests and the oracle's checks take their inputs from here, so that the two
sides see identical samples.

Every generator is deterministic in its seed: a workload id ``cfg`` selects
``numpy.random.SeedSequence(20240325 + cfg)``, spawned once per signal.

Workloads (the paper uses no dataset; these stand in for "a sampled signal
{x_n}, n < N, on [0, T] at interval dt = T/N", Section 2):

* ``tones_real``   -- real sum of sinusoids off the fine grid, Gaussian noise
* ``tones_complex``-- complex unit tones at uniform frequencies, complex noise
* ``precision_tones`` -- complex tones near Nyquist / at irrational multiples of 1/T
* ``uneven_mix``   -- (N, alpha) pairs drawn log-uniformly over 2^a, 3*2^a, 5*2^a
* ``poisson_arrivals`` -- open-loop request arrival times
* ``bin_subset``   -- seeded uniform subset of output bins without replacement
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 20240325


def rngs(cfg: int, count: int):
    """``count`` independent generators for workload ``cfg``."""
    ss = np.random.SeedSequence(BASE_SEED + int(cfg))
    return [np.random.default_rng(s) for s in ss.spawn(int(count))]


def tones_real(rng, N: int, dt: float, alpha: int, ntones: int = 3,
               fmin: float = 5.0, fmax: float = 400.0, amin: float = 0.5,
               amax: float = 2.0, sigma: float = 0.1, offbin: float = 0.1):
    """Real x_n = sum_i A_i sin(2 pi f_i n dt + phi_i) + N(0, sigma^2), float64.

    Each f_i is redrawn until it lies at least ``offbin`` of a fine bin
    (1/(alpha T)) away from every fine bin: frac(f * alpha * T) in
    [offbin, 1 - offbin].  Returns (x, params) with params = (f, A, phi).
    """
    T = N * dt
    f = np.empty(ntones)
    for i in range(ntones):
        while True:
            v = rng.uniform(fmin, fmax)
            fr = (v * alpha * T) % 1.0
            if offbin <= fr <= 1.0 - offbin:
                f[i] = v
                break
    A = rng.uniform(amin, amax, ntones)
    phi = rng.uniform(0.0, 2.0 * math.pi, ntones)
    t = np.arange(N, dtype=np.float64) * dt
    x = np.zeros(N, dtype=np.float64)
    for i in range(ntones):
        x += A[i] * np.sin(2.0 * math.pi * f[i] * t + phi[i])
    x += rng.normal(0.0, sigma, N)
    return x, (f, A, phi)


def tones_complex(rng, N: int, dt: float, ntones: int = 5, sigma: float = 0.05,
                  dtype=np.complex64):
    """Complex x_n = sum_i exp(i(2 pi f_i n dt + phi_i)) + CN(0, sigma^2).

    f_i ~ U[0, 1/dt), phi_i ~ U[0, 2 pi); the noise has independent real and
    imaginary parts, each N(0, sigma^2 / 2).  Synthesised in float64, then
    cast to ``dtype``.
    """
    f = rng.uniform(0.0, 1.0 / dt, ntones)
    phi = rng.uniform(0.0, 2.0 * math.pi, ntones)
    n = np.arange(N, dtype=np.float64)
    x = np.zeros(N, dtype=np.complex128)
    for i in range(ntones):
        # phase reduced in cycles before the 2 pi multiply keeps float64 exact enough
        cyc = np.mod(f[i] * dt * n, 1.0)
        x += np.exp(1j * (2.0 * math.pi * cyc + phi[i]))
    s = sigma / math.sqrt(2.0)
    x += rng.normal(0.0, s, N) + 1j * rng.normal(0.0, s, N)
    return x.astype(dtype)


def precision_tones(rng, N: int, sigma: float = 0.01, dtype=np.complex64):
    """Four unit complex tones placed to stress phase accuracy, plus CN(0, sigma^2).

    Frequencies in units of 1/T: N/2 - (sqrt5-1)/2 (near +Nyquist),
    N-1-(sqrt2-1) (near the sampling rate), N (sqrt3-1) and 1e5*pi (irrational
    multiples of 1/T, folded below N).  Phases uniform.
    """
    cyc_per_T = np.array([N / 2 - (math.sqrt(5) - 1) / 2,
                          N - 1 - (math.sqrt(2) - 1),
                          N * (math.sqrt(3) - 1),
                          1e5 * math.pi])
    cyc_per_T = np.mod(cyc_per_T, N)
    phi = rng.uniform(0.0, 2.0 * math.pi, cyc_per_T.shape[0])
    n = np.arange(N, dtype=np.float64)
    x = np.zeros(N, dtype=np.complex128)
    for i in range(cyc_per_T.shape[0]):
        # cycles at sample n: (f T) * n / N; reduce mod 1 in two exact steps
        k_int = math.floor(cyc_per_T[i])
        k_frac = cyc_per_T[i] - k_int
        cyc = np.mod(np.mod(k_int * n, N) / N + k_frac * n / N, 1.0)
        x += np.exp(1j * (2.0 * math.pi * cyc + phi[i]))
    s = sigma / math.sqrt(2.0)
    x += rng.normal(0.0, s, N) + 1j * rng.normal(0.0, s, N)
    return x.astype(dtype)


def uneven_sizes():
    """The candidate lengths: 2^8..2^18, 3*2^k in [384, 196608], 5*2^k in [320, 163840]."""
    s = [2 ** a for a in range(8, 19)]
    s += [3 * 2 ** a for a in range(7, 17)]
    s += [5 * 2 ** a for a in range(6, 16)]
    return sorted(s)


UNEVEN_ALPHAS = (2, 3, 4, 8, 16)


def uneven_mix(rng, count: int):
    """``count`` (N, alpha) pairs: u ~ U(8, 18), N = the candidate nearest 2^u in
    log2; alpha uniform over {2, 3, 4, 8, 16}."""
    S = np.array(uneven_sizes(), dtype=np.int64)
    logS = np.log2(S.astype(np.float64))
    out = []
    for _ in range(int(count)):
        u = rng.uniform(8.0, 18.0)
        N = int(S[int(np.argmin(np.abs(logS - u)))])
        a = int(UNEVEN_ALPHAS[int(rng.integers(0, len(UNEVEN_ALPHAS)))])
        out.append((N, a))
    return out


def poisson_arrivals(rng, rate_hz: float, count: int):
    """Open-loop arrival times (seconds from 0) of ``count`` requests."""
    gaps = rng.exponential(1.0 / float(rate_hz), int(count))
    return np.cumsum(gaps)


def bin_subset(rng, M: int, k: int):
    """Sorted seeded subset of k bins of [0, M), without replacement (all if M <= k)."""
    if M <= k:
        return np.arange(M, dtype=np.int64)
    return np.sort(rng.choice(M, size=int(k), replace=False)).astype(np.int64)
