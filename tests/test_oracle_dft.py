"""Pins of the direct-DFT oracle (the radix-16 stage prototype's reference):
closed forms of the DFT and the library FFT, which computes the same
transform by a different algorithm."""

import numpy as np

import oracle


def test_delta_and_constant():
    n = 16
    e0 = np.zeros(n, complex)
    e0[0] = 1.0
    assert np.allclose(oracle.dft_direct(e0), np.ones(n), atol=1e-15)
    # shifted delta: a pure phase ramp exp(-2 pi i k m / n)
    em = np.zeros(n, complex)
    em[3] = 1.0
    k = np.arange(n)
    assert np.allclose(oracle.dft_direct(em), np.exp(-2j * np.pi * 3 * k / n), atol=1e-14)
    # constant -> n times a delta at k = 0
    want = np.zeros(n, complex)
    want[0] = n
    assert np.allclose(oracle.dft_direct(np.ones(n, complex)), want, atol=1e-13)


def test_parseval_and_inverse():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((5, 16)) + 1j * rng.standard_normal((5, 16))
    X = oracle.dft_direct(x)
    assert np.allclose(np.sum(np.abs(X) ** 2, -1), 16 * np.sum(np.abs(x) ** 2, -1), rtol=1e-13)
    # F^4 = n^2 I: four rounds of F/4 return the input for n = 16
    assert np.allclose(oracle.dft16_rounds(x, 4), x, atol=1e-13)
    # F^2 x = n x[-m]: two rounds of F/4 reverse the index
    assert np.allclose(oracle.dft16_rounds(x, 2), x[:, (-np.arange(16)) % 16], atol=1e-13)


def test_matches_library_fft():
    rng = np.random.default_rng(4)
    for n in (16, 64, 12):
        x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
        assert np.allclose(oracle.dft_direct(x), np.fft.fft(x, axis=-1), atol=1e-12)


def test_dft_bins_pins():
    # every bin of a short transform equals the DFT-matrix sum
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 64)) + 1j * rng.standard_normal((2, 64))
    assert np.allclose(oracle.dft_bins(x, np.arange(64)), oracle.dft_direct(x), atol=1e-12)
    # inverse of forward: n x (all bins, n = 64)
    X = oracle.dft_bins(x, np.arange(64))
    assert np.allclose(oracle.dft_bins(X, np.arange(64), inverse=True), 64 * x, atol=1e-11)
    # closed forms at a long length, sampled bins: a delta at m gives the
    # phase ramp exp(-2 pi i k m / n), a complex exponential at frequency f
    # gives n at bin f and 0 elsewhere
    n = 1 << 16
    bins = np.array([0, 1, 7, 4097, 30000, n - 1])
    e = np.zeros(n, complex)
    e[12345] = 1.0
    ramp = np.exp(-2j * np.pi * ((bins * 12345) % n) / n)
    assert np.allclose(oracle.dft_bins(e, bins), ramp, atol=1e-12)
    t = np.arange(n)
    tone = np.exp(2j * np.pi * ((4097 * t) % n) / n)
    want = np.where(bins == 4097, n, 0.0)
    assert np.allclose(oracle.dft_bins(tone, bins), want, atol=1e-7)
    # Parseval over all bins at a mid length
    n = 4096
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Y = oracle.dft_bins(y, np.arange(n), block=512)
    assert abs(np.sum(np.abs(Y) ** 2) / (n * np.sum(np.abs(y) ** 2)) - 1) < 1e-12

