"""Direct discrete Fourier transform from its definition (FP64 NumPy): the
reference of the radix-16 stage prototype (a 16-point DFT as a matrix
product against the FFT butterfly).

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
