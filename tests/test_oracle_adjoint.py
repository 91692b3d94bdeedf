"""Pins of the oracle's adjoint: it is the exact vector-Jacobian product of
the propagation, checked against central finite differences (dot-product
test), against the inverse of the linear step (which is unitary), and against
the closed-form derivative of the SPM-only map."""

import math

import numpy as np
import pytest

import oracle
from workloads import Link


def rand_field(rng, n_pol, n, p_w):
    a = rng.standard_normal((n_pol, n)) + 1j * rng.standard_normal((n_pol, n))
    return a * math.sqrt(p_w / n_pol / np.mean(np.abs(a) ** 2))


def real_inner(a, b):
    return float(np.real(np.vdot(a, b)))


@pytest.mark.parametrize("n_pol", [1, 2])
@pytest.mark.parametrize("ase", [False, True])
def test_adjoint_matches_finite_differences(n_pol, ase):
    rng = np.random.default_rng(3 + n_pol)
    n = 256
    ln = Link(n_pol=n_pol, n_samples=n, sample_rate_hz=128e9, span_km=80.0, n_spans=2,
              steps_per_span=6, alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7,
              gamma_per_w_km=1.3, edfa_gain_db=16.0, edfa_nf_db=5.0, ase=ase)
    x = rand_field(rng, n_pol, n, 0.02)         # ~1 rad of nonlinear phase at peaks
    gy = rand_field(rng, n_pol, n, 1.0)         # cotangent dL/dy*
    dx = rand_field(rng, n_pol, n, 0.02)
    # L(x) = 2 Re <gy, y(x)>  =>  dL = 2 Re <gx, dx> with gx = adjoint(gy)
    gx = oracle.adjoint(x, gy, ln, seed=5, realization=1)
    eps = 1e-5
    yp = oracle.propagate(x + eps * dx, ln, seed=5, realization=1)
    ym = oracle.propagate(x - eps * dx, ln, seed=5, realization=1)
    fd = real_inner(gy, (yp - ym) / (2 * eps))
    an = real_inner(gx, dx)
    # central differences: truncation O(eps^2) ~ 1e-10 relative here
    assert abs(fd - an) < 1e-7 * abs(an), (fd, an)


def test_linear_adjoint_is_the_inverse_of_a_lossless_step():
    rng = np.random.default_rng(9)
    ln = Link(n_pol=2, n_samples=512, sample_rate_hz=64e9, span_km=80.0, n_spans=1,
              steps_per_span=10, alpha_db_per_km=0.0, beta2_ps2_per_km=-21.7,
              gamma_per_w_km=0.0)
    x = rand_field(rng, 2, 512, 1.0)
    y = oracle.propagate(x, ln)
    # unitary map: the adjoint maps the output back onto the input
    assert np.allclose(oracle.adjoint(x, y, ln), x, rtol=0, atol=1e-12)


def test_spm_only_adjoint_closed_form():
    # y = x exp(i k |x|^2) (one step, one pol, no loss):
    # dL/dx* = gy e^{-i phi} + 2 k s x,  s = -Im(conj(gy) y)
    rng = np.random.default_rng(4)
    n = 64
    ln = Link(n_pol=1, n_samples=n, sample_rate_hz=64e9, span_km=1.0, n_spans=1,
              steps_per_span=1, alpha_db_per_km=0.0, beta2_ps2_per_km=0.0,
              gamma_per_w_km=100.0)
    x = rand_field(rng, 1, n, 0.005)[0]        # phases ~1 rad
    gy = rand_field(rng, 1, n, 1.0)[0]
    k = 100.0 * 1e-3 * 1e3
    phi = k * np.abs(x) ** 2
    y = x * np.exp(1j * phi)
    want = gy * np.exp(-1j * phi) - 2 * k * np.imag(np.conj(gy) * y) * x
    got = oracle.adjoint(x, gy, ln)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))
