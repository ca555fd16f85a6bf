"""Write the FP64 oracle values of the precision workload on its 16384-bin subset.

Workload: one complex64 signal, N = 2^22 at dt = 1e-3 s (T = 4194.304 s),
alpha = 16 (2^26 bins), siggen.precision_tones with workload seed 2; bins =
siggen.bin_subset(default_rng(2), 2^26, 16384).  Calls only the oracle.
Output: tests/golden/precision_2p22_a16_16384.npz (bins, X as complex128).
Takes a few minutes on 8 cores.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import siggen  # noqa: E402

N, ALPHA, DT, NBINS = 1 << 22, 16, 1e-3, 16384
OUT = os.path.join(HERE, "precision_2p22_a16_16384.npz")


def main():
    x = siggen.precision_tones(siggen.rngs(2, 1)[0], N)
    bins = siggen.bin_subset(np.random.default_rng(2), ALPHA * N, NBINS)
    X = oracle.alpha_dft_bins(x, ALPHA, N * DT, bins)
    np.savez_compressed(OUT, bins=bins, X=X, N=N, alpha=ALPHA, dt=DT)
    print(OUT)


if __name__ == "__main__":
    main()
