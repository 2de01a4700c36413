"""Naive DFTs of the usFFT (oracle side).

Normalisation and sign follow Alg. 1 (step 1&2a and step 2d):
    F[b] = (1/K) sum_{l=0}^{K-1} u_l exp(-2 pi i l b / K).
For real samples F[K-b] = conj(F[b]); both implementations read bin b
through the canonical half-spectrum b' = min(b, K-b) and conjugate when
b > K/2, so that the magnitudes of k and -k are bitwise equal (a reading of
this build, used to make tie handling reproducible).

Pins: a pure tone sampled on its own lattice is one-hot; brute-force tensor
DFT on a tiny full grid; Parseval (tests/test_oracle_dft.py).
"""
import numpy as np


def dft_bins(U, bins):
    """U: (K, G) real samples along the sampling index; bins: (n,) ints in [0, K).
    Returns (n, G) complex coefficients at those bins."""
    U = np.asarray(U, dtype=np.float64)
    K = U.shape[0]
    bins = np.asarray(bins, dtype=np.int64) % K
    canon = np.minimum(bins, K - bins) % K
    l = np.arange(K, dtype=np.int64)
    phase = (canon[:, None] * l[None, :]) % K
    E = np.exp(-2j * np.pi * phase / K)
    F = (E @ U) / K
    flip = bins > K - bins
    F[flip] = np.conj(F[flip])
    return F
