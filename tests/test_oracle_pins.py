"""Pins of the FP64 oracle against results fixed by physics and mathematics.

Each test checks the oracle against something other than itself: an analytic
solution of the propagation equation, a conservation law, a textbook link
budget rule, or an independent implementation of a published generator.
Together they are chosen so that a plausible slip in the oracle (a wrong
sign or unit of beta2, alpha in dB instead of nepers, a missing 1/2, the
wrong Manakov factor, sigma instead of sigma/sqrt(2), a shifted RNG counter)
fails at least one of them.
"""

import math
import os

import numpy as np
import pytest

import oracle
from workloads import Link

SSMF = dict(alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7, gamma_per_w_km=1.3)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _link(**kw):
    base = dict(n_pol=1, n_samples=1024, sample_rate_hz=64e9, span_km=80.0,
                n_spans=1, steps_per_span=80, **SSMF)
    base.update(kw)
    return Link(**base)


# --------------------------------------------------------------------------
# T1: dispersion + loss only, against the analytic Gaussian-pulse solution
# --------------------------------------------------------------------------

def gaussian_solution(t, t0, beta2, z, alpha_db_per_km):
    """Unchirped Gaussian under the linear equation dA/dz = -i(beta2/2)A_TT:
    A(z,T) = T0 / sqrt(T0^2 - i beta2 z) exp(-T^2 / (2 (T0^2 - i beta2 z))),
    times the field loss 10^(-alpha_dB z_km / 20) (Agrawal, ch. 3, Gaussian
    pulses)."""
    q = t0 ** 2 - 1j * beta2 * z
    loss = 10.0 ** (-alpha_db_per_km * (z / 1e3) / 20.0)
    return loss * t0 / np.sqrt(q) * np.exp(-t ** 2 / (2.0 * q))


@pytest.mark.parametrize("beta2", [-21.7, 16.0])
@pytest.mark.parametrize("n_spans,steps", [(1, 80), (3, 7)])
def test_t1_dispersion_matches_gaussian_closed_form(beta2, n_spans, steps):
    n, fs = 2048, 64e9
    dt = 1.0 / fs
    t0 = 4 * dt
    t = (np.arange(n) - n // 2) * dt
    a0 = np.exp(-t ** 2 / (2 * t0 ** 2)).astype(np.complex128)
    ln = _link(n_samples=n, sample_rate_hz=fs, n_spans=n_spans,
               steps_per_span=steps, gamma_per_w_km=0.0, beta2_ps2_per_km=beta2)
    out = oracle.propagate(a0, ln)
    z = 80e3 * n_spans
    want = gaussian_solution(t, t0, beta2 * 1e-27, z, 0.2)
    assert rel(out, want) < 1e-12


def test_t1_wrong_beta2_sign_is_detected():
    # the closed form distinguishes the sign convention of beta2
    n, fs = 2048, 64e9
    dt = 1.0 / fs
    t0 = 4 * dt
    t = (np.arange(n) - n // 2) * dt
    a0 = np.exp(-t ** 2 / (2 * t0 ** 2)).astype(np.complex128)
    ln = _link(n_samples=n, sample_rate_hz=fs, gamma_per_w_km=0.0)
    out = oracle.propagate(a0, ln)
    flipped = gaussian_solution(t, t0, +21.7e-27, 80e3, 0.2)
    assert rel(out, flipped) > 1e-2


# --------------------------------------------------------------------------
# T2: nonlinearity + loss only, against the exact SPM rotation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n_pol", [1, 2])
@pytest.mark.parametrize("steps", [1, 5, 80])
def test_t2_spm_matches_effective_length(n_pol, steps):
    rng = np.random.default_rng(7)
    n = 512
    a0 = (rng.standard_normal((n_pol, n)) + 1j * rng.standard_normal((n_pol, n))) * 0.05
    ln = _link(n_pol=n_pol, n_samples=n, steps_per_span=steps, beta2_ps2_per_km=0.0)
    out = oracle.propagate(a0, ln)
    # L_eff = (1 - 10^(-alpha_dB L / 10)) / (alpha_dB ln10 / 10): power decay
    # integrated over the span, written directly in dB units
    l_km = 80.0
    leff_km = (1 - 10 ** (-0.2 * l_km / 10)) / (0.2 * math.log(10) / 10)
    assert abs(leff_km - 21.169) < 1e-3
    c = 1.0 if n_pol == 1 else 8.0 / 9.0
    ptot = np.sum(np.abs(a0) ** 2, axis=0)
    want = a0 * 10 ** (-0.2 * l_km / 20) * np.exp(1j * c * 1.3 * leff_km * ptot)
    assert rel(out, want) < 1e-12


def test_t2_phase_adds_over_transparent_spans():
    rng = np.random.default_rng(8)
    n = 256
    a0 = (rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))) * 0.05
    ln = _link(n_pol=2, n_samples=n, n_spans=4, steps_per_span=10,
               beta2_ps2_per_km=0.0, edfa_gain_db=16.0)
    out = oracle.propagate(a0, ln)
    leff_km = (1 - 10 ** (-1.6)) / (0.2 * math.log(10) / 10)
    ptot = np.sum(np.abs(a0) ** 2, axis=0)
    want = a0 * np.exp(1j * (8 / 9) * 1.3 * leff_km * 4 * ptot)
    assert rel(out, want) < 1e-12


# --------------------------------------------------------------------------
# T3: power conservation (alpha = 0) and exact loss (alpha > 0)
# --------------------------------------------------------------------------

def _qam_like(rng, n_pol, n, p_w):
    a = rng.standard_normal((n_pol, n)) + 1j * rng.standard_normal((n_pol, n))
    return a * math.sqrt(p_w / n_pol / np.mean(np.abs(a) ** 2))


@pytest.mark.parametrize("n_pol", [1, 2])
def test_t3_power_conserved_without_loss(n_pol):
    rng = np.random.default_rng(9)
    a0 = _qam_like(rng, n_pol, 1024, 0.02)
    ln = _link(n_pol=n_pol, alpha_db_per_km=0.0, steps_per_span=40)
    # check after every span of a 5-span link, step by step through resume
    a = a0
    e0 = np.sum(np.abs(a0) ** 2)
    for s in range(5):
        a = oracle.propagate(a, ln.replace(n_spans=5), span_begin=s, span_end=s + 1)
        assert abs(np.sum(np.abs(a) ** 2) / e0 - 1) < 1e-13


def test_t3_power_decays_by_span_loss():
    rng = np.random.default_rng(10)
    a0 = _qam_like(rng, 2, 1024, 0.02)
    ln = _link(n_pol=2)
    out = oracle.propagate(a0, ln)
    ratio = np.sum(np.abs(out) ** 2) / np.sum(np.abs(a0) ** 2)
    assert abs(ratio / 10 ** (-1.6) - 1) < 1e-13  # 80 km x 0.2 dB/km = 16 dB


# --------------------------------------------------------------------------
# T4: the fundamental soliton, with second-order step convergence
# --------------------------------------------------------------------------

def soliton_case(n_pol, steps, theta=0.3):
    n, fs = 1024, 128e9
    dt = 1.0 / fs
    t0 = 8 * dt
    beta2 = -21.7e-27
    gamma = 1.3e-3
    c = 1.0 if n_pol == 1 else 8.0 / 9.0
    p0 = abs(beta2) / (c * gamma * t0 ** 2)      # soliton order N = 1
    t = (np.arange(n) - n // 2) * dt
    env = np.sqrt(p0) / np.cosh(t / t0)
    if n_pol == 1:
        a0 = env[None, :].astype(np.complex128)
    else:
        a0 = np.stack([math.cos(theta) * env, math.sin(theta) * env]).astype(np.complex128)
    ld = t0 ** 2 / abs(beta2)
    n_spans = 4
    ln = Link(n_pol=n_pol, n_samples=n, sample_rate_hz=fs, span_km=80.0,
              n_spans=n_spans, steps_per_span=steps, alpha_db_per_km=0.0,
              beta2_ps2_per_km=-21.7, gamma_per_w_km=1.3)
    z = 80e3 * n_spans
    want = a0 * np.exp(1j * c * gamma * p0 * z / 2.0)
    return a0, ln, want, z / ld


@pytest.mark.parametrize("n_pol", [1, 2])
def test_t4_soliton_second_order_convergence(n_pol):
    errs = []
    for steps in (10, 20, 40):
        a0, ln, want, zld = soliton_case(n_pol, steps)
        assert zld > 1.5   # the test propagates over more than one dispersion length
        errs.append(rel(oracle.propagate(a0, ln), want))
    s1 = math.log2(errs[0] / errs[1])
    s2 = math.log2(errs[1] / errs[2])
    assert 1.9 < s1 < 2.1 and 1.9 < s2 < 2.1, errs
    assert errs[-1] < 1e-3


def test_t4_soliton_fine_steps_is_accurate():
    a0, ln, want, _ = soliton_case(2, 400)
    assert rel(oracle.propagate(a0, ln), want) < 2e-5


def test_t4_wrong_manakov_factor_breaks_the_soliton():
    a0, ln, want, _ = soliton_case(2, 200)
    bad = oracle.propagate(a0, ln.replace(nl_factor=1.0))
    assert rel(bad, want) > 1e-2


# --------------------------------------------------------------------------
# T5: time reversal (the merged symmetric scheme is a palindrome)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n_pol", [1, 2])
def test_t5_time_reversal(n_pol):
    rng = np.random.default_rng(11)
    a0 = _qam_like(rng, n_pol, 1024, 0.01)
    ln = _link(n_pol=n_pol, n_spans=2, steps_per_span=13)
    out = oracle.propagate(a0, ln)
    back = oracle.propagate(out, ln.replace(alpha_db_per_km=-0.2,
                                            beta2_ps2_per_km=21.7,
                                            gamma_per_w_km=-1.3))
    assert rel(back, a0) < 1e-12
    assert rel(out, a0) > 1e-1


# --------------------------------------------------------------------------
# T7: the noise generator against an independent Philox4x64-10
# --------------------------------------------------------------------------

M64 = (1 << 64) - 1


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds written from its published definition
    (Salmon et al., SC'11): per round two 64x64->128 multiplications, a
    word permutation, xor with the key; the key advances by the Weyl
    constants between rounds."""
    m0, m1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
    w0, w1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
    x = list(ctr)
    k0, k1 = key
    for r in range(10):
        if r:
            k0, k1 = (k0 + w0) & M64, (k1 + w1) & M64
        p0 = m0 * x[0]
        p1 = m1 * x[2]
        x = [(p1 >> 64) ^ x[1] ^ k0, p1 & M64, (p0 >> 64) ^ x[3] ^ k1, p0 & M64]
    return x


@pytest.mark.parametrize("seed,real,span", [(0, 0, 0), (1002, 3, 9),
                                            (M64, 70000, 65535)])
def test_t7_noise_words_follow_philox_definition(seed, real, span):
    words = oracle.ase_words(seed, real, span, 40)
    key = (seed & M64, (real * 65536 + span) & M64)
    for t in (0, 1, 2, 17, 39):
        assert [int(v) for v in words[t]] == philox4x64_10((t, 0, 0, 0), key)


def test_t7_uniforms_are_exact_in_single_precision():
    w = np.array([0, 1 << 41, M64, 12345678901234567890], dtype=np.uint64)
    u = oracle.uniform_from_words(w)
    assert u.min() > 0 and u.max() < 1
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    assert u[0] == 0.5 * 2 ** -23 and u[2] == 1 - 0.5 * 2 ** -23


# --------------------------------------------------------------------------
# T8: ASE statistics and the textbook OSNR rule
# --------------------------------------------------------------------------

def _ase_link(n_spans, n=1 << 14, n_pol=2):
    return Link(n_pol=n_pol, n_samples=n, sample_rate_hz=128e9, span_km=80.0,
                n_spans=n_spans, steps_per_span=4, alpha_db_per_km=0.2,
                beta2_ps2_per_km=-21.7, gamma_per_w_km=0.0,
                edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True)


def test_t8_osnr_rule_of_thumb():
    """OSNR in 0.1 nm (12.5 GHz) ~= 58 dB + P_ch[dBm] - NF - span loss
    - 10 log10(N_spans) at 1550 nm (standard link-budget rule, noise summed
    over both polarisations, G ~ G - 1)."""
    n_spans = 3
    ln = _ase_link(n_spans, n=1 << 16)
    out = oracle.propagate(np.zeros((2, ln.n_samples), complex), ln, seed=5)
    p_ase = np.sum(np.mean(np.abs(out) ** 2, axis=1))     # both pols, over fs
    p_ref = p_ase * 12.5e9 / ln.sample_rate_hz
    osnr_db = 10 * math.log10(1e-3 / p_ref)               # for a 0 dBm channel
    rule = 58.0 - 5.0 - 16.0 - 10 * math.log10(n_spans)
    # the rule rounds 57.96 dB to 58 and uses G for G - 1 (0.11 dB)
    assert abs(osnr_db - rule) < 0.25, (osnr_db, rule)


def test_t8_ase_is_circular_white_gaussian():
    from scipy import stats
    ln = _ase_link(1)
    out = oracle.propagate(np.zeros((2, ln.n_samples), complex), ln, seed=77)
    sigma2 = out.real.var() + out.imag.var()
    for q in range(2):
        x = out[q]
        s = math.sqrt(sigma2 / 2)
        assert abs(x.real.mean()) < 5 * s / math.sqrt(x.size)
        assert abs(x.imag.mean()) < 5 * s / math.sqrt(x.size)
        assert abs(x.real.var() / x.imag.var() - 1) < 0.06
        assert abs(np.mean(x.real * x.imag)) < 5 * s * s / math.sqrt(x.size)
        assert stats.kstest(x.real / s, "norm").pvalue > 1e-4
    # independence of the two polarisations and flat spectrum
    c = np.vdot(out[0], out[1]) / np.sqrt(np.vdot(out[0], out[0]).real
                                          * np.vdot(out[1], out[1]).real)
    assert abs(c) < 5 / math.sqrt(ln.n_samples)
    spec = np.abs(np.fft.fft(out[0])) ** 2
    bands = spec.reshape(16, -1).mean(axis=1)
    assert bands.max() / bands.min() < 1.2


def test_t8_variance_grows_linearly_over_transparent_spans():
    one = _ase_link(1)
    four = _ase_link(4)
    z = np.zeros((2, one.n_samples), complex)
    v1 = np.mean(np.abs(oracle.propagate(z, one, seed=3)) ** 2)
    v4 = np.mean(np.abs(oracle.propagate(z, four, seed=3)) ** 2)
    assert abs(v4 / v1 / 4 - 1) < 0.05


def test_t8_noise_depends_on_seed_realisation_and_span():
    p = oracle.si_params(_ase_link(2, n=256))
    a = oracle.ase_noise(p, 1, 0, 0)
    for other in (oracle.ase_noise(p, 2, 0, 0), oracle.ase_noise(p, 1, 1, 0),
                  oracle.ase_noise(p, 1, 0, 1)):
        assert not np.allclose(a, other)
    assert np.array_equal(a, oracle.ase_noise(p, 1, 0, 0))


# --------------------------------------------------------------------------
# Resume: propagating span by span equals one call
# --------------------------------------------------------------------------

def test_span_resume_is_bitwise():
    rng = np.random.default_rng(12)
    ln = _link(n_pol=2, n_samples=512, n_spans=3, steps_per_span=5,
               edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True)
    a0 = _qam_like(rng, 2, 512, 0.002)
    whole = oracle.propagate(a0, ln, seed=9, realization=4)
    part = oracle.propagate(a0, ln, seed=9, realization=4, span_end=1)
    part = oracle.propagate(part, ln, seed=9, realization=4, span_begin=1)
    assert np.array_equal(whole, part)


def _kat_rows():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "philox4x64_10_kat.txt")
    rows = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_t7_philox_known_answer_vectors():
    # the published known-answer vectors pin the Philox definition used by
    # the independent implementation above and the oracle's noise words
    rows = _kat_rows()
    assert len(rows) == 2
    for ctr, key, want in rows:
        assert list(philox4x64_10(ctr, key)) == want
    # oracle: key (seed, realisation 2^16 + span) = (0, 0), counter 0
    words = oracle.ase_words(0, 0, 0, 1)
    assert [int(v) for v in np.asarray(words).reshape(-1)[:4]] == rows[0][2]
