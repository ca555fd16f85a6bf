"""FP64 CPU oracle for the alpha-dense DFT -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it.

It evaluates the definition of the transform directly (paper, Section 2:
eq. (7) first line on the grid of eq. (6), with the T/N forward factor of
eq. (2), sign convention of Section 3):

    X_m = (T/N) * sum_{n<N} x_n * exp(-2 pi i m n / (alpha N)),  m < alpha N

in double precision, one output bin at a time (``dd_oracle.c``), and the
inverse transform (eq. (7) second line, read with the 1/(alpha T) factor that
undoes the forward one):

    x_n = (1/(alpha T)) * sum_{m<alpha N} X_m * exp(+2 pi i m n / (alpha N)),  n < N

Pins: every function here is checked against facts the paper and the
mathematics fix, in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dd_oracle.c")
_LIB = os.path.join(_HERE, "libdd_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP).  Returns the .so path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.dd_oracle_bins_mut.argtypes = [dp, dp, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_double, ip, ctypes.c_int64,
                                           dp, dp, ctypes.c_int]
        lib.dd_oracle_bins_mut.restype = ctypes.c_int
        lib.dd_oracle_inv_mut.argtypes = [dp, dp, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_double, ip, ctypes.c_int64,
                                          dp, dp, ctypes.c_int]
        lib.dd_oracle_inv_mut.restype = ctypes.c_int
        lib.dd_oracle_threads.argtypes = []
        lib.dd_oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads() -> int:
    """Number of OpenMP threads the oracle uses."""
    return int(_load().dd_oracle_threads())


def alpha_dft_bins(x, alpha: int, T: float, bins, *, mutation: int = 0) -> np.ndarray:
    """X_m for the requested bins m (int array, each in [0, alpha*N)).

    ``x`` is the stored signal (real or complex, any float precision); it is
    promoted exactly to complex128 before use.  Returns complex128.
    ``mutation`` != 0 plants a known mistake (for the pin self-test only).
    """
    xa = np.asarray(x)
    if xa.ndim != 1:
        raise ValueError("x must be 1-D")
    N = xa.shape[0]
    xr = np.ascontiguousarray(xa.real, dtype=np.float64)
    xi = (np.ascontiguousarray(xa.imag, dtype=np.float64) if np.iscomplexobj(xa)
          else np.zeros(N, dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(bins, dtype=np.int64).reshape(-1))
    outr = np.empty(b.shape[0], dtype=np.float64)
    outi = np.empty(b.shape[0], dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    rc = _load().dd_oracle_bins_mut(
        xr.ctypes.data_as(dp), xi.ctypes.data_as(dp), N, int(alpha), float(T),
        b.ctypes.data_as(ip), b.shape[0], outr.ctypes.data_as(dp),
        outi.ctypes.data_as(dp), int(mutation))
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    return outr + 1j * outi


def alpha_dft(x, alpha: int, T: float, *, mutation: int = 0) -> np.ndarray:
    """The full alpha-dense spectrum, all alpha*N bins in natural order."""
    N = np.asarray(x).shape[0]
    return alpha_dft_bins(x, alpha, T, np.arange(alpha * N, dtype=np.int64),
                          mutation=mutation)


def inverse_alpha_dft_samples(X, alpha: int, T: float, samples, *, mutation: int = 0) -> np.ndarray:
    """x_n of the inverse transform for the requested samples n (each in
    [0, alpha*N), N = len(X) / alpha).  ``X`` is promoted exactly to
    complex128; returns complex128.  ``mutation`` != 0 plants a known
    mistake (for the pin self-test only)."""
    Xa = np.asarray(X)
    if Xa.ndim != 1 or Xa.shape[0] % int(alpha):
        raise ValueError("X must be 1-D with alpha*N entries")
    N = Xa.shape[0] // int(alpha)
    Xr = np.ascontiguousarray(Xa.real, dtype=np.float64)
    Xi = (np.ascontiguousarray(Xa.imag, dtype=np.float64) if np.iscomplexobj(Xa)
          else np.zeros(Xa.shape[0], dtype=np.float64))
    n = np.ascontiguousarray(np.asarray(samples, dtype=np.int64).reshape(-1))
    outr = np.empty(n.shape[0], dtype=np.float64)
    outi = np.empty(n.shape[0], dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    rc = _load().dd_oracle_inv_mut(
        Xr.ctypes.data_as(dp), Xi.ctypes.data_as(dp), N, int(alpha), float(T),
        n.ctypes.data_as(ip), n.shape[0], outr.ctypes.data_as(dp),
        outi.ctypes.data_as(dp), int(mutation))
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (rc={rc})")
    return outr + 1j * outi


def inverse_alpha_dft(X, alpha: int, T: float, *, mutation: int = 0) -> np.ndarray:
    """All N samples of the inverse transform, n = 0 .. N-1."""
    N = np.asarray(X).shape[0] // int(alpha)
    return inverse_alpha_dft_samples(X, alpha, T, np.arange(N, dtype=np.int64), mutation=mutation)


def decimated_dft(x, p: int, T: float, *, mutation: int = 0) -> np.ndarray:
    """The transform for alpha = 1/p (p a positive divisor of N; Section 2, the
    case alpha < 1): X_m = (T/N) sum_{n<N} x_n exp(-2 pi i m n / (N/p)),
    m < N/p.  Since exp(-2 pi i m n p / N) is the alpha = 1 kernel at bin p m,
    the definition is evaluated as the alpha = 1 sum at bins p m.  Returns
    complex128."""
    N = np.asarray(x).shape[0]
    if p < 1 or N % p:
        raise ValueError("p must be a positive divisor of N")
    return alpha_dft_bins(x, 1, T, np.arange(N // p, dtype=np.int64) * p, mutation=mutation)
