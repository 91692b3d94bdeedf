"""Plain FP64 oracle of learned digital back-propagation (NumPy, complex128).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.

Learned digital back-propagation (Haeger and Pfister, "Physics-based deep
learning for fiber-optic communication systems", IEEE J. Sel. Areas Commun.
39(1), 2021) is a split-step back-propagation whose linear steps are short
complex FIR filters and whose nonlinear steps are Kerr phase rotations with a
trainable coefficient; all of them are fitted by gradient descent on a
symbol-domain loss.  The formulation here, per realisation and K steps
k = 0..K-1 over a field x in C^{P x N} (P polarisations, N samples,
circular time axis):

    FIR        y_p[n] = sum_{t=0}^{T-1} h_k[t] x_p[(n + c - t) mod N],
               c = (T - 1) / 2, the same taps for every polarisation
    nonlinear  x_p[n] <- y_p[n] exp(i xi_k sum_q |y_q[n]|^2)

The output z is x after the K steps.  Loss: a real matched filter g of
2R + 1 taps (g[j + R], j = -R..R) sampled at the symbol instants,

    u_p[m] = sum_j g[j + R] z_p[(sps m - j) mod N],
    L      = mean over (b, p, m) of |u_p[m] - s_p[m]|^2.

Gradients follow PyTorch's complex convention: for a complex quantity w the
returned gradient is dL/dRe w + i dL/dIm w (= 2 dL/dw*); for the real xi it
is dL/dxi.  With that convention and the output cotangent gz of a step:

    phi   = xi sum_q |y_q|^2,   z = y exp(i phi)
    s     = -Im sum_q conj(gz_q) z_q              (per sample)
    dL/dxi  += sum_n |y[n]|^2 s[n]                (|y|^2 summed over q)
    gy    = gz exp(-i phi) + 2 xi s y
    gh[t] += sum_{p,n} gy_p[n] conj(x_p[(n + c - t) mod N])
    gx[m] = sum_t conj(h[t]) gy[(m - c + t) mod N]

(the pullbacks of z = y exp(i xi |y|^2), which is holomorphic in neither y
nor xi, and of the circular convolution).  The step structure and these
formulas are written from the definitions above; nothing is blocked, fused
or reordered.

The initial parameters ``init_params`` come from the link: step k
back-propagates 1/S of a span (S steps per span, from the last span to the
first) with the truncated impulse response of the inverse dispersion as
taps (the least-squares T-tap fit of that response over the full band),
scaled by the peak gain of the truncated filter, and the midpoint-weighted
nonlinear coefficient of the forward model with the opposite sign.  The
scaling is a reading of ours: a truncated all-pass response ripples above
unit gain at some frequencies (1.33 for 15 taps over 40 km at 128 GS/s), and
K cascaded steps would amplify those by the K-th power (285 for K = 20),
noise and rounding included; scaled, every step is contractive.  When T
covers the whole circular response the filter is all-pass and the scale is
one.
"""

from __future__ import annotations

import math

import numpy as np

from .ssfm_ref import angular_frequency, nl_step_length, si_params

__all__ = ["fir", "nl_rotate", "ldbp_forward", "matched_filter_samples",
           "mse_loss", "mse_grad", "ldbp_backward", "init_params"]


def _as3(a: np.ndarray) -> np.ndarray:
    """[B, P, N] view of a [P, N] or [B, P, N] field."""
    a = np.asarray(a, dtype=np.complex128)
    return a[None] if a.ndim == 2 else a


def fir(x: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """y[n] = sum_t taps[t] x[(n + c - t) mod N] along the last axis."""
    taps = np.asarray(taps, dtype=np.complex128)
    c = (taps.size - 1) // 2
    y = np.zeros_like(x, dtype=np.complex128)
    for t in range(taps.size):
        # np.roll(x, s)[n] = x[n - s]; s = t - c gives x[n + c - t]
        y += taps[t] * np.roll(x, t - c, axis=-1)
    return y


def nl_rotate(y: np.ndarray, xi: float) -> np.ndarray:
    """y_p exp(i xi sum_q |y_q|^2); polarisation axis -2."""
    pw = np.sum(np.abs(y) ** 2, axis=-2, keepdims=True)
    return y * np.exp(1j * xi * pw)


def ldbp_forward(x: np.ndarray, taps: np.ndarray, xi: np.ndarray,
                 keep: bool = False):
    """Apply the K steps to a [P, N] or [B, P, N] field.  With ``keep`` also
    return the tape [(x_k, y_k)] of every step's FIR input and output."""
    a = np.array(x, dtype=np.complex128)
    tape = []
    for k in range(len(xi)):
        y = fir(a, taps[k])
        if keep:
            tape.append((a, y))
        a = nl_rotate(y, float(xi[k]))
    return (a, tape) if keep else a


def matched_filter_samples(z: np.ndarray, mf: np.ndarray, sps: int) -> np.ndarray:
    """u[m] = sum_j mf[j + R] z[(sps m - j) mod N], m = 0..N/sps - 1."""
    mf = np.asarray(mf, dtype=np.float64)
    r = (mf.size - 1) // 2
    acc = np.zeros_like(z, dtype=np.complex128)
    for j in range(-r, r + 1):
        acc += mf[j + r] * np.roll(z, j, axis=-1)   # z[n - j]
    return acc[..., ::sps]


def mse_loss(z: np.ndarray, symbols: np.ndarray, mf: np.ndarray, sps: int) -> float:
    """mean |u - s|^2 over every realisation, polarisation and symbol."""
    u = matched_filter_samples(z, mf, sps)
    return float(np.mean(np.abs(u - np.asarray(symbols)) ** 2))


def mse_grad(z: np.ndarray, symbols: np.ndarray, mf: np.ndarray, sps: int) -> np.ndarray:
    """Gradient of ``mse_loss`` w.r.t. z (PyTorch convention)."""
    u = matched_filter_samples(z, mf, sps)
    du = 2.0 * (u - np.asarray(symbols)) / u.size
    up = np.zeros_like(z, dtype=np.complex128)
    up[..., ::sps] = du
    mf = np.asarray(mf, dtype=np.float64)
    r = (mf.size - 1) // 2
    g = np.zeros_like(z, dtype=np.complex128)
    for j in range(-r, r + 1):
        # gz[n] = sum_m mf[sps m - n + R] du[m] = sum_j mf[j + R] up[n + j]
        g += mf[j + r] * np.roll(up, -j, axis=-1)
    return g


def ldbp_backward(x: np.ndarray, taps: np.ndarray, xi: np.ndarray,
                  grad_out: np.ndarray):
    """Vector-Jacobian product of ``ldbp_forward``: given the gradient of the
    output, return (grad_x, grad_taps [K, T], grad_xi [K])."""
    squeeze = np.asarray(x).ndim == 2
    _, tape = ldbp_forward(_as3(x), taps, xi, keep=True)
    g = np.array(_as3(grad_out), dtype=np.complex128)
    taps = np.asarray(taps, dtype=np.complex128)
    n_steps, n_taps = taps.shape
    c = (n_taps - 1) // 2
    g_taps = np.zeros((n_steps, n_taps), dtype=np.complex128)
    g_xi = np.zeros(n_steps, dtype=np.float64)
    for k in reversed(range(n_steps)):
        xk, yk = tape[k]
        pw = np.sum(np.abs(yk) ** 2, axis=-2, keepdims=True)
        rot = np.exp(1j * xi[k] * pw)
        zk = yk * rot
        s = -np.imag(np.sum(np.conj(g) * zk, axis=-2, keepdims=True))
        g_xi[k] = float(np.sum(pw * s))
        gy = g * np.conj(rot) + 2.0 * xi[k] * s * yk
        for t in range(n_taps):
            g_taps[k, t] = np.sum(gy * np.conj(np.roll(xk, t - c, axis=-1)))
        g = np.zeros_like(gy)
        for t in range(n_taps):
            g += np.conj(taps[k, t]) * np.roll(gy, c - t, axis=-1)   # gy[m - c + t]
    return (g[0] if squeeze else g), g_taps, g_xi


def init_params(link, n_taps: int, steps_per_span: int):
    """Taps [K, T] and coefficients [K] for K = n_spans * steps_per_span,
    from the link (see the module docstring)."""
    p = si_params(link)
    n, fs = p["n"], p["fs"]
    hd = p["span_m"] / steps_per_span
    omega = angular_frequency(n, fs)
    # inverse of the forward linear phase exp(i (beta2/2) omega^2 h)
    resp = np.exp(-1j * 0.5 * p["beta2"] * omega ** 2 * hd)
    ir = np.fft.ifft(resp)
    c = (n_taps - 1) // 2
    base = np.array([ir[(t - c) % n] for t in range(n_taps)])
    # peak gain of the truncated filter on the n-point grid
    kernel = np.zeros(n, dtype=np.complex128)
    for t in range(n_taps):
        kernel[(t - c) % n] += base[t]
    base = base / np.max(np.abs(np.fft.fft(kernel)))
    gspan = math.sqrt(p["gain"]) * math.exp(-p["alpha"] * p["span_m"] / 2.0)
    k_total = p["n_spans"] * steps_per_span
    taps = np.empty((k_total, n_taps), dtype=np.complex128)
    xi = np.empty(k_total, dtype=np.float64)
    hnl = nl_step_length(p["alpha"], hd)
    for k in range(k_total):
        j = k % steps_per_span          # sub-step within the span, from its end
        taps[k] = base / gspan if j == 0 else base
        z_mid = p["span_m"] - (j + 0.5) * hd
        xi[k] = -p["c_nl"] * p["gamma"] * hnl * math.exp(-p["alpha"] * z_mid)
    return taps, xi

