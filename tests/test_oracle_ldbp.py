"""Pins of the learned-DBP oracle against what the mathematics fixes: the FIR
is a circular convolution (FFT route), the nonlinear step a pure phase (SPM
closed form), the matched filter a circular convolution sampled at the
symbol instants; the gradients match central finite differences and
PyTorch's own autograd of the forward definition; the initial parameters
undo the oracle's forward propagation on a link they can represent."""

import math

import numpy as np
import pytest

import oracle
from workloads import Link
from workloads.signals import rrc_taps


def rand_c(rng, *shape, scale=1.0):
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def padded(taps, n):
    """Length-n circular kernel with taps[t] at offset t - c."""
    c = (len(taps) - 1) // 2
    k = np.zeros(n, dtype=np.complex128)
    for t, v in enumerate(taps):
        k[(t - c) % n] += v
    return k


def real_inner(a, b):
    return float(np.real(np.vdot(a, b)))


def test_fir_is_circular_convolution():
    rng = np.random.default_rng(1)
    x = rand_c(rng, 2, 2, 64)
    h = rand_c(rng, 15)
    want = np.fft.ifft(np.fft.fft(x, axis=-1) * np.fft.fft(padded(h, 64)), axis=-1)
    np.testing.assert_allclose(oracle.fir(x, h), want, rtol=0, atol=1e-12)


def test_fir_delta_and_shift_are_exact():
    rng = np.random.default_rng(2)
    x = rand_c(rng, 2, 33)
    d = np.zeros(15, dtype=np.complex128)
    d[7] = 1.0
    assert np.array_equal(oracle.fir(x, d), x)
    d = np.zeros(15, dtype=np.complex128)
    d[8] = 1.0                        # y[n] = x[n - 1]
    assert np.array_equal(oracle.fir(x, d), np.roll(x, 1, axis=-1))


def test_spm_only_closed_form():
    # identity taps: |y| is invariant, so the K rotations add up
    rng = np.random.default_rng(3)
    x = rand_c(rng, 3, 2, 40, scale=0.3)
    k = 5
    taps = np.zeros((k, 15), dtype=np.complex128)
    taps[:, 7] = 1.0
    xi = rng.uniform(-2.0, 2.0, size=k)
    pw = np.sum(np.abs(x) ** 2, axis=-2, keepdims=True)
    want = x * np.exp(1j * np.sum(xi) * pw)
    np.testing.assert_allclose(oracle.ldbp_forward(x, taps, xi), want, rtol=0, atol=1e-12)


def test_linear_only_is_product_of_responses():
    rng = np.random.default_rng(4)
    x = rand_c(rng, 2, 128)
    k = 4
    taps = rand_c(rng, k, 15, scale=0.3)
    resp = np.ones(128, dtype=np.complex128)
    for t in taps:
        resp = resp * np.fft.fft(padded(t, 128))
    want = np.fft.ifft(np.fft.fft(x, axis=-1) * resp, axis=-1)
    got = oracle.ldbp_forward(x, taps, np.zeros(k))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.max(np.abs(want)))


def test_matched_filter_is_sampled_convolution():
    rng = np.random.default_rng(5)
    z = rand_c(rng, 2, 2, 256)
    g = rrc_taps(2, 0.1, 20)
    full = np.fft.ifft(np.fft.fft(z, axis=-1) * np.fft.fft(padded(g, 256)), axis=-1)
    np.testing.assert_allclose(oracle.matched_filter_samples(z, g, 2), full[..., ::2],
                               rtol=0, atol=1e-12)


def test_loss_with_unit_filter():
    rng = np.random.default_rng(6)
    z = rand_c(rng, 2, 2, 64)
    s = z[..., ::2].copy()
    assert oracle.mse_loss(z, s, np.ones(1), 2) == 0.0
    s2 = rand_c(rng, 2, 2, 32)
    assert math.isclose(oracle.mse_loss(z, s2, np.ones(1), 2),
                        float(np.mean(np.abs(z[..., ::2] - s2) ** 2)), rel_tol=1e-14)


def test_rrc_taps_nyquist():
    # RRC convolved with itself is a raised cosine: zero at nonzero symbol
    # instants (up to the truncation of the long tails)
    g = rrc_taps(4, 0.25, 4 * 40)
    rc = np.convolve(g, g)
    mid = rc.size // 2
    assert abs(rc[mid] - 1.0) < 1e-12
    for m in range(1, 6):
        assert abs(rc[mid + 4 * m]) < 2e-3


def test_mse_grad_finite_differences():
    rng = np.random.default_rng(7)
    z = rand_c(rng, 2, 2, 64)
    s = rand_c(rng, 2, 2, 32)
    g = rrc_taps(2, 0.1, 9)
    dz = rand_c(rng, 2, 2, 64)
    eps = 1e-3      # quadratic: no truncation error at any step, so take a large one
    fd = (oracle.mse_loss(z + eps * dz, s, g, 2) - oracle.mse_loss(z - eps * dz, s, g, 2)) / (2 * eps)
    an = real_inner(oracle.mse_grad(z, s, g, 2), dz)
    # rounding of the O(1) loss values: ~1e-16 / eps relative to |an|
    assert abs(fd - an) < 1e-10 * abs(an)


def _problem(seed, b=2, p=2, n=48, k=4):
    rng = np.random.default_rng(seed)
    x = rand_c(rng, b, p, n, scale=0.5)
    taps = rand_c(rng, k, 15, scale=0.15)
    taps[:, 7] += 1.0
    xi = rng.uniform(-1.5, 1.5, size=k)
    return rng, x, taps, xi


@pytest.mark.parametrize("p", [1, 2])
def test_backward_finite_differences(p):
    rng, x, taps, xi = _problem(11 + p, p=p)
    gz = rand_c(rng, *x.shape)
    gx, gtaps, gxi = oracle.ldbp_backward(x, taps, xi, gz)

    def L(x_, taps_, xi_):
        # a linear functional of the output: its gradient w.r.t. z is gz
        return real_inner(gz, oracle.ldbp_forward(x_, taps_, xi_))

    # fourth-order central differences: the taps enter through K cascaded
    # convolutions and Kerr phases, so the second-order truncation error
    # (eps^2 times the third derivative over 6) would be ~1e-7 relative at
    # eps = 1e-6; the fourth-order error at eps = 1e-5 is ~1e-10 here
    def fd4(f, eps=1e-5):
        return (f(-2 * eps) - 8 * f(-eps) + 8 * f(eps) - f(2 * eps)) / (12 * eps)

    dx = rand_c(rng, *x.shape)
    fd = fd4(lambda e: L(x + e * dx, taps, xi))
    assert abs(fd - real_inner(gx, dx)) < 1e-8 * abs(fd)
    dt = rand_c(rng, *taps.shape)
    fd = fd4(lambda e: L(x, taps + e * dt, xi))
    assert abs(fd - real_inner(gtaps, dt)) < 1e-8 * abs(fd)
    dxi = rng.standard_normal(xi.shape)
    fd = fd4(lambda e: L(x, taps, xi + e * dxi))
    assert abs(fd - float(np.dot(gxi, dxi))) < 1e-8 * abs(fd)


def test_backward_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng, x, taps, xi = _problem(21, b=2, p=2, n=40, k=3)
    s = rand_c(rng, 2, 2, 20)
    g = rrc_taps(2, 0.1, 6)
    r = (g.size - 1) // 2

    tx = torch.tensor(x, requires_grad=True)
    tt = torch.tensor(taps, requires_grad=True)
    txi = torch.tensor(xi, requires_grad=True)
    a = tx
    c = 7
    for k in range(len(xi)):
        y = sum(tt[k, t] * torch.roll(a, t - c, dims=-1) for t in range(15))
        pw = torch.sum(torch.abs(y) ** 2, dim=-2, keepdim=True)
        a = y * torch.exp(1j * txi[k] * pw)
    u = sum(float(g[j + r]) * torch.roll(a, j, dims=-1) for j in range(-r, r + 1))[..., ::2]
    loss = torch.mean(torch.abs(u - torch.tensor(s)) ** 2)
    loss.backward()

    z = oracle.ldbp_forward(x, taps, xi)
    assert math.isclose(oracle.mse_loss(z, s, g, 2), float(loss.detach()), rel_tol=1e-12)
    gz = oracle.mse_grad(z, s, g, 2)
    gx, gtaps, gxi = oracle.ldbp_backward(x, taps, xi, gz)
    np.testing.assert_allclose(gx, tx.grad.numpy(), rtol=0, atol=1e-12 * np.max(np.abs(gx)))
    np.testing.assert_allclose(gtaps, tt.grad.numpy(), rtol=0, atol=1e-12 * np.max(np.abs(gtaps)))
    np.testing.assert_allclose(gxi, txi.grad.numpy(), rtol=0, atol=1e-12 * np.max(np.abs(gxi)))


def _short_link(gamma):
    # N = T = 15: the taps cover every circular offset once, so the initial
    # filter is the whole impulse response of the inverse dispersion
    return Link(n_pol=2, n_samples=15, sample_rate_hz=128e9, span_km=80.0, n_spans=3,
                steps_per_span=40, alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7,
                gamma_per_w_km=gamma, edfa_gain_db=14.0, edfa_nf_db=5.0, ase=False)


def test_init_params_invert_linear_link():
    # loss, dispersion and a gain that does not compensate the loss: the
    # back-propagation is the exact inverse of the oracle's linear steps
    rng = np.random.default_rng(31)
    ln = _short_link(0.0)
    x = rand_c(rng, 2, 15, scale=1e-2)
    rx = oracle.propagate(x, ln)
    taps, xi = oracle.init_params(ln, 15, 2)
    back = oracle.ldbp_forward(rx, taps, xi)
    err = np.linalg.norm(back - x) / np.linalg.norm(x)
    assert err < 1e-12, err


def test_init_params_nonlinear_coefficients():
    # ~1 mW: the Kerr phase is compensated in sign and size -- the initial
    # coefficients beat linear-only back-propagation, the opposite sign and
    # half or twice their size
    rng = np.random.default_rng(32)
    ln = _short_link(1.3)
    x = rand_c(rng, 2, 15, scale=math.sqrt(1e-3 / 2))
    rx = oracle.propagate(x, ln)
    taps, xi = oracle.init_params(ln, 15, 2)

    def err(scale):
        return np.linalg.norm(oracle.ldbp_forward(rx, taps, scale * xi) - x)

    e1 = err(1.0)
    assert e1 < 0.35 * err(0.0)
    assert e1 < err(-1.0) and e1 < err(0.5) and e1 < err(2.0)
