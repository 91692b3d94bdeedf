"""Transmitted-field synthesis: 16-QAM, root-raised-cosine shaping, WDM.

Every function is seeded and deterministic.  Fields are returned as
``complex128`` arrays of shape ``[n_pol, n_samples]``; the time-average of
``sum_p |A_p|^2`` equals the launch power in watts (split equally over the
polarisations, and per channel for WDM).
"""

from __future__ import annotations

import math
from typing import Optional

import numpy as np

__all__ = ["dbm_to_watt", "qam16_symbols", "rrc_response", "rrc_taps",
           "shaped_field", "dual_pol_field", "wdm_field", "make_field",
           "field_and_targets"]


def dbm_to_watt(p_dbm: float) -> float:
    return 1e-3 * 10.0 ** (p_dbm / 10.0)


def qam16_symbols(rng: np.random.Generator, n: int) -> np.ndarray:
    """``n`` uniform 16-QAM symbols on {+-1, +-3}^2, scaled to unit energy."""
    levels = np.array([-3.0, -1.0, 1.0, 3.0])
    i = rng.integers(0, 4, size=n)
    q = rng.integers(0, 4, size=n)
    return (levels[i] + 1j * levels[q]) / math.sqrt(10.0)


def rrc_response(f: np.ndarray, symbol_rate: float, rolloff: float) -> np.ndarray:
    """Frequency response of the root-raised-cosine filter (unit passband)."""
    a = np.abs(np.asarray(f, dtype=np.float64))
    f1 = (1.0 - rolloff) * symbol_rate / 2.0
    f2 = (1.0 + rolloff) * symbol_rate / 2.0
    out = np.zeros_like(a)
    out[a <= f1] = 1.0
    band = (a > f1) & (a <= f2)
    if rolloff > 0:
        out[band] = np.sqrt(0.5 * (1.0 + np.cos(
            math.pi / (rolloff * symbol_rate) * (a[band] - f1))))
    return out


def rrc_taps(sps: int, rolloff: float, half: int) -> np.ndarray:
    """Real root-raised-cosine matched filter of 2 half + 1 taps at ``sps``
    samples per symbol, t = j / sps symbols, unit energy (closed form of the
    RRC impulse response; the removable singularities at t = 0 and
    |t| = 1 / (4 rolloff) take their limits)."""
    b = rolloff
    out = np.empty(2 * half + 1)
    for i, j in enumerate(range(-half, half + 1)):
        t = j / sps
        if j == 0:
            v = 1.0 + b * (4.0 / math.pi - 1.0)
        elif b > 0 and abs(abs(4.0 * b * t) - 1.0) < 1e-12:
            v = (b / math.sqrt(2.0)) * ((1 + 2 / math.pi) * math.sin(math.pi / (4 * b))
                                        + (1 - 2 / math.pi) * math.cos(math.pi / (4 * b)))
        else:
            num = math.sin(math.pi * t * (1 - b)) + 4 * b * t * math.cos(math.pi * t * (1 + b))
            den = math.pi * t * (1 - (4 * b * t) ** 2)
            v = num / den
        out[i] = v
    return out / math.sqrt(np.sum(out ** 2))


def shaped_field(symbols: np.ndarray, sps: int, symbol_rate: float,
                 rolloff: float) -> np.ndarray:
    """Zero-insertion upsampling by ``sps`` and circular RRC shaping."""
    n = symbols.size * sps
    up = np.zeros(n, dtype=np.complex128)
    up[::sps] = symbols
    fs = symbol_rate * sps
    f = np.fft.fftfreq(n, d=1.0 / fs)
    return np.fft.ifft(np.fft.fft(up) * rrc_response(f, symbol_rate, rolloff))


def _normalise(a: np.ndarray, p_watt: float) -> np.ndarray:
    """Scale each polarisation to ``p_watt / n_pol`` mean power."""
    n_pol = a.shape[0]
    pw = np.mean(np.abs(a) ** 2, axis=-1, keepdims=True)
    return a * np.sqrt((p_watt / n_pol) / pw)


def dual_pol_field(rng: np.random.Generator, n_pol: int, n_samples: int,
                   sps: int, symbol_rate: float, rolloff: float,
                   launch_dbm: float) -> np.ndarray:
    """Single-carrier field with independent symbols per polarisation."""
    if n_samples % sps:
        raise ValueError("n_samples must be a multiple of sps")
    m = n_samples // sps
    a = np.stack([shaped_field(qam16_symbols(rng, m), sps, symbol_rate, rolloff)
                  for _ in range(n_pol)])
    return _normalise(a, dbm_to_watt(launch_dbm))


def field_and_targets(rng: np.random.Generator, n_pol: int, n_samples: int,
                      sps: int, symbol_rate: float, rolloff: float,
                      launch_dbm: float, mf: np.ndarray):
    """Single-carrier field (as ``dual_pol_field``) and its symbols in field
    units: each polarisation's symbols times the power normalisation of that
    polarisation and the gain of the real matched filter ``mf`` (2R + 1 taps)
    on one shaped pulse, so that the matched filter sampled at the symbol
    instants returns the targets up to intersymbol interference.  Returns
    (field [P, N], targets [P, N / sps])."""
    if n_samples % sps:
        raise ValueError("n_samples must be a multiple of sps")
    m = n_samples // sps
    syms = np.stack([qam16_symbols(rng, m) for _ in range(n_pol)])
    raw = np.stack([shaped_field(syms[p], sps, symbol_rate, rolloff) for p in range(n_pol)])
    pw = np.mean(np.abs(raw) ** 2, axis=-1, keepdims=True)
    scale = np.sqrt((dbm_to_watt(launch_dbm) / n_pol) / pw)
    impulse = np.zeros(m, dtype=np.complex128)
    impulse[0] = 1.0
    pulse = shaped_field(impulse, sps, symbol_rate, rolloff)
    r = (len(mf) - 1) // 2
    gain = sum(mf[j + r] * pulse[(-j) % n_samples] for j in range(-r, r + 1))
    return raw * scale, syms * scale * gain


def wdm_field(rng: np.random.Generator, n_pol: int, n_samples: int,
              sample_rate: float, n_channels: int, spacing: float,
              symbol_rate: float, rolloff: float,
              launch_dbm_per_channel: float) -> np.ndarray:
    """``n_channels`` carriers centred on 0 Hz, independent symbols per
    channel and polarisation, each channel at the same launch power."""
    sps = int(round(sample_rate / symbol_rate))
    if abs(sps * symbol_rate - sample_rate) > 1e-6 * sample_rate:
        raise ValueError("sample rate must be an integer multiple of the symbol rate")
    t = np.arange(n_samples) / sample_rate
    out = np.zeros((n_pol, n_samples), dtype=np.complex128)
    for c in range(n_channels):
        fc = (c - (n_channels - 1) / 2.0) * spacing
        base = dual_pol_field(rng, n_pol, n_samples, sps, symbol_rate, rolloff,
                              launch_dbm_per_channel)
        out += base * np.exp(2j * math.pi * fc * t)
    return out


def make_field(workload, seed: Optional[int] = None) -> np.ndarray:
    """Transmitted field of a :class:`workloads.configs.Workload`."""
    rng = np.random.default_rng(workload.symbol_seed if seed is None else seed)
    ln = workload.link
    if workload.n_channels > 1:
        return wdm_field(rng, ln.n_pol, ln.n_samples, ln.sample_rate_hz,
                         workload.n_channels, workload.channel_spacing_hz,
                         workload.symbol_rate_hz, workload.rolloff,
                         workload.launch_dbm)
    return dual_pol_field(rng, ln.n_pol, ln.n_samples, workload.sps,
                          workload.symbol_rate_hz, workload.rolloff,
                          workload.launch_dbm)
