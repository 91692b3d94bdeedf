"""The seeded input generators: power, spectrum and determinism."""

import math

import numpy as np
import pytest

from workloads import (CONFIGS, batch_config, dbm_to_watt, make_field,
                       qam16_symbols, rrc_response)


def test_qam16_alphabet_and_energy():
    s = qam16_symbols(np.random.default_rng(0), 1 << 16)
    levels = np.unique(np.round(s.real * math.sqrt(10)))
    assert list(levels) == [-3, -1, 1, 3]
    assert abs(np.mean(np.abs(s) ** 2) - 1) < 0.02


def test_rrc_squared_is_raised_cosine_nyquist():
    # |H_rrc|^2 summed with its copy shifted by the symbol rate is flat
    rs, beta = 32e9, 0.1
    f = np.linspace(0, rs, 1001)
    h2 = rrc_response(f, rs, beta) ** 2 + rrc_response(f - rs, rs, beta) ** 2
    assert np.allclose(h2, 1.0, atol=1e-12)
    assert rrc_response(np.array([0.56 * rs]), rs, beta)[0] == 0


@pytest.mark.parametrize("cfg", [1, 2, 5])
def test_launch_power_and_band_limit(cfg):
    w = CONFIGS[cfg]
    a = make_field(w)
    ln = w.link
    assert a.shape == (ln.n_pol, ln.n_samples) and a.dtype == np.complex128
    assert abs(np.mean(np.sum(np.abs(a) ** 2, axis=0)) / dbm_to_watt(w.launch_dbm) - 1) < 1e-12
    f = np.fft.fftfreq(ln.n_samples, 1 / ln.sample_rate_hz)
    spec = np.abs(np.fft.fft(a, axis=-1)) ** 2
    out = np.abs(f) > (1 + w.rolloff) * w.symbol_rate_hz / 2 + 1e-3
    assert spec[:, out].sum() < 1e-20 * spec.sum()


def test_wdm_carriers_on_exact_bins_and_power():
    w = CONFIGS[3]
    ln = w.link
    df = ln.sample_rate_hz / ln.n_samples
    assert (w.channel_spacing_hz / df) == int(w.channel_spacing_hz / df)
    a = make_field(w)
    assert abs(np.mean(np.sum(np.abs(a) ** 2, axis=0)) / (5 * 1e-3) - 1) < 0.05
    f = np.fft.fftfreq(ln.n_samples, 1 / ln.sample_rate_hz)
    spec = np.sum(np.abs(np.fft.fft(a, axis=-1)) ** 2, axis=0)
    for c in range(5):
        fc = (c - 2) * 75e9
        band = np.abs(f - fc) < 0.5 * 64e9 * 1.1 / 1
        assert spec[band].sum() > 0.19 * spec.sum()


def test_generators_are_deterministic():
    a = make_field(CONFIGS[1])
    b = make_field(CONFIGS[1])
    assert np.array_equal(a, b)
    assert not np.array_equal(a, make_field(CONFIGS[1], seed=1))


def test_batch_config_ranges():
    items = batch_config()
    assert len(items) == 256
    assert {it.n_samples for it in items} <= {1 << k for k in range(12, 17)}
    assert all(-4 <= it.launch_dbm <= 6 and 1 <= it.n_spans <= 10 for it in items)
    assert len({it.seed for it in items}) == 256
