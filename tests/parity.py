"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare it with the FP64 oracle on the same seeded inputs.

Tolerances (FP32 path, complex64 output):
  * full spectrum checked: relative L2 error <= 1e-5 (the stated bound);
  * sampled bins: RMS error over the sample divided by the RMS of the whole
    spectrum <= 1e-5 (an unbiased estimate of the full-spectrum relative L2;
    the whole-spectrum RMS is exact from the input by Parseval, eq. (8):
    rms(X) = (T/N) sqrt(sum_n |x_n|^2), see spectrum_rms);
  * every checked bin m within 2e-5 rms(X) + 1e-5 |X_m|.
FP64 path (complex128): 1e-12, and 1e-11 rms(X) + 1e-12 |X_m| per bin.
The element bound follows from FP32 rounding in the transform: the error of
a bin has a part spread over the spectrum, of about eps*sqrt(log2 M)*rms(X)
(eps = 2^-24, below 5e-7 rms(X) for M <= 2^31), and a part proportional to
the values it is computed from, since twiddle and butterfly rounding scale
with them; for tonal signals those concentrate at the peaks, where |X_m| is
up to sqrt(N) times rms(X), so the second part is bounded relative to
|X_m| (a few eps there; 1e-5 leaves a wide margin).  Either way a wrong
twiddle or index (an error of order |X_m| or rms(X)) fails it.  The relative
L2 over a random bin subset is NOT used as a sampled bound: for tonal
signals most random bins lie far below the spectrum RMS, which inflates it
30-90x even for a textbook FP32 FFT.
"""
import numpy as np

TOL = {"f32": (1e-5, 2e-5), "f64": (1e-12, 1e-11)}


def rel_l2(got, ref):
    ref = np.asarray(ref)
    return float(np.linalg.norm(np.asarray(got) - ref) / max(np.linalg.norm(ref), 1e-300))


def spectrum_rms(x, T):
    """RMS of |X_m| over all alpha*N bins, from the input alone (Parseval,
    eq. (8)): sum_m |X_m|^2 = (T/N)^2 alpha N sum_n |x_n|^2, so
    rms = (T/N) sqrt(sum_n |x_n|^2), independent of alpha."""
    x = np.asarray(x).astype(np.complex128)
    return float(T / x.shape[-1] * np.sqrt(np.sum(np.abs(x) ** 2)))


def assert_close(got, ref, kind, what="", full_rms=None):
    """Full-spectrum check when full_rms is None; sampled check otherwise."""
    rl, el = TOL[kind]
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    if ref.size == 0:
        return 0.0
    err = np.abs(got - ref)
    if full_rms is None:
        r = rel_l2(got, ref)
        scale = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
        assert r <= rl, f"{what}: rel L2 {r:.3e} > {rl:.1e}"
    else:
        scale = float(full_rms)
        r = float(np.sqrt(np.mean(err ** 2))) / max(scale, 1e-300)
        assert r <= rl, f"{what}: sampled rms err / spectrum rms {r:.3e} > {rl:.1e}"
    bound = el * max(scale, 1e-300) + rl * np.abs(ref)
    worst = int(np.argmax(err - bound))
    assert err[worst] <= bound[worst], (f"{what}: bin {worst} err {err[worst]:.3e} > {el:.1e} * rms {scale:.3e} "
                                        f"+ {rl:.1e} * |X| {abs(ref[worst]):.3e}")
    return r


def assert_same(got, ref, what=""):
    """Two FP32 results of the whole spectrum (e.g. one signal run by two
    paths): each is within the FP32 bound of the exact spectrum, so they are
    compared with the same full-spectrum check."""
    return assert_close(got, ref, "f32", what)


def gpu_alpha_dft(x_np, alpha, T, flags=0):
    """Run the library on a [batch, N] (or [N]) numpy array; returns numpy."""
    import torch
    import paper_2403_16665_amd as dd
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to("cuda")
    X = dd.alpha_dft(x, alpha, T, flags=flags)
    torch.cuda.synchronize()
    return X.cpu().numpy()
