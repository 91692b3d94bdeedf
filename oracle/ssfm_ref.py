"""Plain FP64 split-step Fourier oracle (NumPy, complex128).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.

The paper this library accompanies states no fibre-propagation model; every
formula below is textbook fibre optics, cited to its source:

* Propagation equation (Agrawal, *Nonlinear Fiber Optics*, ch. 2, the
  nonlinear Schroedinger equation with loss), per polarisation p::

      dA_p/dz = -(alpha/2) A_p - i (beta2/2) d^2A_p/dT^2
                + i c_nl gamma (sum_q |A_q|^2) A_p

  with c_nl = 1 for one polarisation and 8/9 for two (the Manakov-PMD
  average, Marcuse, Menyuk and Wai, J. Lightwave Technol. 15(9), 1997).
* Symmetric split-step Fourier method (Agrawal, ch. 2, split-step Fourier
  method): per span of n steps of length h, half a linear step, then
  n - 1 times (nonlinear step, full linear step), a last nonlinear step and
  a last half linear step.  Adjacent half steps are merged.
* Nonlinear step length h_nl = 2 sinh(alpha h / 2) / alpha: the integral of
  the power decay exp(-alpha z) over the step, taken about its midpoint, so
  that the nonlinear-only case telescopes to the effective length
  L_eff = (1 - exp(-alpha L)) / alpha for any n.
* Lumped amplifier at the end of every span: field gain sqrt(G) and
  amplified spontaneous emission of one-sided spectral density
  n_sp (G - 1) h nu per polarisation with n_sp = NF / 2 (high-gain form of
  the noise figure; Desurvire, *Erbium-Doped Fiber Amplifiers*), white over
  the simulated bandwidth fs, independent per polarisation and quadrature.
* Noise draws: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11), taken
  from NumPy's implementation, and the Box-Muller transform (Box and
  Muller, 1958).  Key = (seed, realisation * 2^16 + span); the block with
  counter value t (t = time-sample index) gives the four words
  (w0, w1, w2, w3); polarisation x uses (w0, w1), polarisation y (w2, w3).
  A word w maps to u = ((w >> 41) + 1/2) 2^-23, exactly representable in
  single and double precision, and g = sqrt(-2 ln u1) exp(2 pi i u2).

FFT sign and normalisation conventions do not matter: the linear factor
depends on omega only through omega^2.
"""

from __future__ import annotations

import math
from typing import Optional

import numpy as np

__all__ = ["si_params", "angular_frequency", "linear_factor",
           "nl_step_length", "linear_step", "nl_step", "ase_words",
           "uniform_from_words", "ase_noise", "edfa", "propagate",
           "propagate_batch", "nl_pullback", "adjoint"]

PLANCK = 6.62607015e-34          # J s (SI exact)
DEFAULT_CARRIER_HZ = 193.4145e12  # 1550 nm


def si_params(link) -> dict:
    """Convert a link in quoted units to SI.

    alpha [1/m] is the power attenuation in nepers: dB/km * ln(10)/10 / 1e3.
    beta2 [s^2/m] = ps^2/km * 1e-24 / 1e3.  gamma [1/(W m)] = 1/(W km) / 1e3.
    """
    n_pol = int(link.n_pol)
    c_nl = link.nl_factor
    if c_nl is None or (isinstance(c_nl, float) and math.isnan(c_nl)):
        c_nl = 1.0 if n_pol == 1 else 8.0 / 9.0
    carrier = link.carrier_hz
    if carrier is None or (isinstance(carrier, float) and math.isnan(carrier)):
        carrier = DEFAULT_CARRIER_HZ
    span_m = link.span_km * 1e3
    return dict(
        n_pol=n_pol,
        n=int(link.n_samples),
        fs=float(link.sample_rate_hz),
        alpha=link.alpha_db_per_km * math.log(10.0) / 10.0 / 1e3,
        beta2=link.beta2_ps2_per_km * 1e-24 / 1e3,
        gamma=link.gamma_per_w_km / 1e3,
        c_nl=float(c_nl),
        span_m=span_m,
        n_spans=int(link.n_spans),
        steps=int(link.steps_per_span),
        h=span_m / int(link.steps_per_span),
        gain=10.0 ** (link.edfa_gain_db / 10.0),
        nf=10.0 ** (link.edfa_nf_db / 10.0),
        ase=bool(link.ase),
        carrier=float(carrier),
    )


def angular_frequency(n: int, fs: float) -> np.ndarray:
    """omega_k = 2 pi f_k on the FFT grid of n points at sample rate fs."""
    return 2.0 * math.pi * np.fft.fftfreq(n, d=1.0 / fs)


def linear_factor(beta2: float, alpha: float, omega: np.ndarray,
                  length: float) -> np.ndarray:
    """Exact frequency-domain solution of the linear part over ``length``:
    exp(i (beta2/2) omega^2 length - alpha length / 2)."""
    return np.exp(1j * (beta2 / 2.0) * omega ** 2 * length - alpha * length / 2.0)


def nl_step_length(alpha: float, h: float) -> float:
    """h_nl = 2 sinh(alpha h / 2) / alpha (h when alpha = 0)."""
    if alpha == 0.0:
        return h
    return 2.0 * math.sinh(alpha * h / 2.0) / alpha


def linear_step(a: np.ndarray, factor: np.ndarray) -> np.ndarray:
    """A <- IFFT(factor * FFT(A)) along the time axis, every polarisation."""
    return np.fft.ifft(factor * np.fft.fft(a, axis=-1), axis=-1)


def nl_step(a: np.ndarray, coef: float) -> np.ndarray:
    """A_p <- A_p exp(i coef sum_q |A_q|^2) (exact solution of the
    nonlinear part, which leaves every |A_p| unchanged)."""
    power = np.sum(np.abs(a) ** 2, axis=0, keepdims=True)
    return a * np.exp(1j * coef * power)


def ase_words(seed: int, realization: int, span: int, n: int) -> np.ndarray:
    """Philox4x64-10 blocks for counters 0..n-1 under key
    (seed, realization * 2^16 + span), shape [n, 4] of uint64.

    NumPy's generator advances its counter before producing a block, so the
    stream is started from counter 2^256 - 1 to make block t carry counter t.
    """
    m64 = (1 << 64) - 1
    key = np.array([seed & m64, (realization * 65536 + span) & m64],
                   dtype=np.uint64)
    ctr = np.array([m64, m64, m64, m64], dtype=np.uint64)
    gen = np.random.Philox(counter=ctr, key=key)
    return gen.random_raw(4 * n).astype(np.uint64).reshape(n, 4)


def uniform_from_words(w: np.ndarray) -> np.ndarray:
    """u = ((w >> 41) + 1/2) * 2^-23, in (0, 1)."""
    return ((w >> np.uint64(41)).astype(np.float64) + 0.5) * 2.0 ** -23


def ase_noise(p: dict, seed: int, realization: int, span: int) -> np.ndarray:
    """ASE field added after span ``span``: (sigma / sqrt 2)(g1 + i g2) per
    polarisation with sigma^2 = n_sp (G - 1) h nu fs."""
    n_pol, n = p["n_pol"], p["n"]
    sigma2 = (p["nf"] / 2.0) * (p["gain"] - 1.0) * PLANCK * p["carrier"] * p["fs"]
    w = ase_words(seed, realization, span, n)
    out = np.empty((n_pol, n), dtype=np.complex128)
    for q in range(n_pol):
        u1 = uniform_from_words(w[:, 2 * q])
        u2 = uniform_from_words(w[:, 2 * q + 1])
        g = np.sqrt(-2.0 * np.log(u1)) * np.exp(2j * math.pi * u2)
        out[q] = math.sqrt(sigma2 / 2.0) * g
    return out


def edfa(a: np.ndarray, p: dict, seed: int, realization: int,
         span: int) -> np.ndarray:
    """Lumped amplifier: A <- sqrt(G) A (+ ASE when enabled and G > 1)."""
    a = a * math.sqrt(p["gain"])
    if p["ase"] and p["gain"] > 1.0:
        a = a + ase_noise(p, seed, realization, span)
    return a


def propagate(field, link, seed: int = 0, realization: int = 0,
              span_begin: int = 0, span_end: Optional[int] = None) -> np.ndarray:
    """Propagate ``field`` ([n_pol, n] or [n]) through spans
    ``span_begin .. span_end - 1`` of ``link``; returns complex128."""
    p = si_params(link)
    a = np.array(field, dtype=np.complex128)
    squeeze = a.ndim == 1
    if squeeze:
        a = a[None, :]
    if a.shape != (p["n_pol"], p["n"]):
        raise ValueError(f"field shape {a.shape} does not match the link "
                         f"({p['n_pol']}, {p['n']})")
    span_end = p["n_spans"] if span_end is None else span_end
    omega = angular_frequency(p["n"], p["fs"])
    h = p["h"]
    half = linear_factor(p["beta2"], p["alpha"], omega, h / 2.0)
    full = linear_factor(p["beta2"], p["alpha"], omega, h)
    coef = p["c_nl"] * p["gamma"] * nl_step_length(p["alpha"], h)
    amplified = p["gain"] != 1.0 or p["ase"]
    for s in range(span_begin, span_end):
        a = linear_step(a, half)
        for j in range(p["steps"]):
            a = nl_step(a, coef)
            a = linear_step(a, full if j < p["steps"] - 1 else half)
        if amplified:
            a = edfa(a, p, seed, realization, s)
    return a[0] if squeeze else a


def propagate_batch(fields, link, seed: int = 0, realization0: int = 0,
                    span_begin: int = 0, span_end: Optional[int] = None):
    """Realisation ``b`` of a [B, n_pol, n] batch uses noise key
    (seed, realization0 + b)."""
    fields = np.asarray(fields)
    return np.stack([propagate(fields[b], link, seed, realization0 + b,
                               span_begin, span_end)
                     for b in range(fields.shape[0])])


# ---------------------------------------------------------------------------
# Adjoint (vector-Jacobian product) of the propagation, for gradients.
#
# For a real loss L and the conjugate Wirtinger derivatives g = dL/dA*, each
# step of the scheme is pulled back exactly:
#   linear step  y = ifft(H fft(x)):   g_x = ifft(conj(H) fft(g_y))
#   nonlinear    y_p = x_p exp(i phi), phi = coef sum_q |x_q|^2:
#                g_x_p = g_y_p exp(-i phi) + 2 s coef x_p,
#                s = -Im(sum_q conj(g_y_q) y_q)
#   amplifier    y = sqrt(G) x + noise:  g_x = sqrt(G) g_y
# (chain rule on y(x, x*); the noise does not depend on the field).  The
# forward states are stored, step by step, and the pullbacks applied in
# reverse order.  The map from g_y to g_x is real-linear, so any constant
# scaling of the incoming cotangent (e.g. PyTorch's factor 2) passes through.
# ---------------------------------------------------------------------------

def nl_pullback(x: np.ndarray, gy: np.ndarray, coef: float) -> np.ndarray:
    power = np.sum(np.abs(x) ** 2, axis=0, keepdims=True)
    rot = np.exp(1j * coef * power)
    y = x * rot
    s = -np.imag(np.sum(np.conj(gy) * y, axis=0, keepdims=True))
    return gy * np.conj(rot) + 2.0 * s * coef * x


def adjoint(field, grad_out, link, seed: int = 0, realization: int = 0) -> np.ndarray:
    """dL/dA_in* given dL/dA_out* for propagate(field, link, seed, realization)."""
    p = si_params(link)
    a = np.array(field, dtype=np.complex128)
    g = np.array(grad_out, dtype=np.complex128)
    squeeze = a.ndim == 1
    if squeeze:
        a, g = a[None, :], g[None, :]
    omega = angular_frequency(p["n"], p["fs"])
    h = p["h"]
    half = linear_factor(p["beta2"], p["alpha"], omega, h / 2.0)
    full = linear_factor(p["beta2"], p["alpha"], omega, h)
    coef = p["c_nl"] * p["gamma"] * nl_step_length(p["alpha"], h)
    amplified = p["gain"] != 1.0 or p["ase"]
    # forward, keeping the input of every nonlinear step
    tape = []
    for s in range(p["n_spans"]):
        a = linear_step(a, half)
        for j in range(p["steps"]):
            tape.append(a)
            a = nl_step(a, coef)
            a = linear_step(a, full if j < p["steps"] - 1 else half)
        if amplified:
            a = edfa(a, p, seed, realization, s)
    # reverse
    k = len(tape)
    for s in reversed(range(p["n_spans"])):
        if amplified:
            g = g * math.sqrt(p["gain"])
        for j in reversed(range(p["steps"])):
            g = linear_step(g, np.conj(full if j < p["steps"] - 1 else half))
            k -= 1
            g = nl_pullback(tape[k], g, coef)
        g = linear_step(g, np.conj(half))
    return g[0] if squeeze else g
