"""Direct discrete Fourier transform from its definition (FP64 NumPy): the
reference of the radix-16 stage prototype (a 16-point DFT as a matrix
product against the FFT butterfly) and of the library's transform stages
(selected bins of long transforms, ``dft_bins``).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path.

    X[k] = sum_n x[n] exp(-2 pi i n k / N),  k, n = 0 .. N - 1

written as the O(N^2) sum over the DFT matrix, with no factorisation.
"""

import numpy as np


def dft_matrix(n: int) -> np.ndarray:
    """F[k, m] = exp(-2 pi i k m / n), complex128."""
    k = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(k, k) / n)


def dft_direct(x: np.ndarray) -> np.ndarray:
    """DFT along the last axis by the direct sum."""
    x = np.asarray(x, dtype=np.complex128)
    return x @ dft_matrix(x.shape[-1]).T


def dft16_rounds(x: np.ndarray, rounds: int) -> np.ndarray:
    """(F / 4)^rounds applied to every length-16 row of x."""
    y = np.asarray(x, dtype=np.complex128)
    assert y.shape[-1] == 16
    for _ in range(rounds):
        y = dft_direct(y) / 4.0
    return y


def dft_bins(x: np.ndarray, bins, inverse: bool = False, block: int = 64) -> np.ndarray:
    """X[..., k] = sum_n x[..., n] exp(-+2 pi i n k / N) for the listed bins k
    (the sign + for inverse; unnormalised), by the direct sum over n.  The
    exponent n k is reduced modulo N in integers first (the DFT kernel is
    N-periodic in n k), so every angle is formed from an index below N."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    bins = np.asarray(bins, dtype=np.int64)
    sign = 1.0 if inverse else -1.0
    t = np.arange(n, dtype=np.int64)
    out = np.empty(x.shape[:-1] + (bins.size,), dtype=np.complex128)
    for b0 in range(0, bins.size, block):
        kb = bins[b0:b0 + block]
        m = np.outer(kb, t) % n
        w = np.exp(sign * 2j * np.pi * m / n)
        out[..., b0:b0 + kb.size] = x @ w.T
    return out

