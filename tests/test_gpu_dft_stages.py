"""The library's transform stages alone (ssfm_dft through the C ABI) against
the DFT's definition (oracle.dft_bins, the direct sum): the LDS-resident
transform and the four-step column and row passes, forward and inverse, on
sampled bins (every bin for short lengths), with the four-step path's
frequency order (bin k1 + n1 k2 at position k1 n2 + k2)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from fieldcheck import check
from workloads import Link

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_03509_amd as m
    m.load_library()
    return m


def link(n_pol, n):
    return Link(n_pol=n_pol, n_samples=n, sample_rate_hz=128e9, span_km=80.0, n_spans=1,
                steps_per_span=1, alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7,
                gamma_per_w_km=1.3)


def storage_of_bins(plan_info, n, bins):
    """Position of bin k in the transform's output."""
    if plan_info["path"] == 1:
        return bins
    n1, n2 = plan_info["n1"], plan_info["n2"]
    return (bins % n1) * n2 + bins // n1


def sampled_bins(rng, n):
    if n <= 4096:
        return np.arange(n)
    return np.unique(np.concatenate([[0, 1, n // 2, n - 1], rng.integers(0, n, 253)]))


CASES = [(64, 1, 2), (4096, 2, 2), (8192, 1, 2), (8192, 2, 2), (1 << 14, 2, 3),
         (1 << 15, 1, 3), (1 << 16, 2, 3), (1 << 16, 2, 40), (1 << 18, 2, 5)]


@pytest.mark.parametrize("n,n_pol,batch", CASES)
def test_forward_transform_matches_direct_dft(ssfm, n, n_pol, batch):
    print(f"case n={n} n_pol={n_pol} batch={batch}", flush=True)
    rng = np.random.default_rng(n + n_pol + batch)
    x = (rng.standard_normal((batch, n_pol, n)) + 1j * rng.standard_normal((batch, n_pol, n)))
    x = x.astype(np.complex64)
    plan = ssfm.Plan(link(n_pol, n))
    try:
        t = torch.from_numpy(x).cuda()
        ssfm.ssfm_dft(plan.handle, t, inverse=False)
        torch.cuda.synchronize()
        got = t.cpu().numpy().astype(np.complex128)
        info = plan.info
    finally:
        plan.close()
    bins = sampled_bins(rng, n)
    pos = storage_of_bins(info, n, bins)
    for b in sorted({0, batch - 1}):
        want = oracle.dft_bins(x[b].astype(np.complex128), bins)
        check(got[b][:, pos], want, 1e-6, what=f"realisation {b}")


@pytest.mark.parametrize("n,n_pol,batch", [(4096, 2, 2), (8192, 2, 1), (1 << 14, 2, 3),
                                           (1 << 16, 2, 40), (1 << 18, 1, 2)])
def test_inverse_transform_matches_direct_dft(ssfm, n, n_pol, batch):
    print(f"case n={n} n_pol={n_pol} batch={batch}", flush=True)
    rng = np.random.default_rng(7 * n + n_pol)
    # a spectrum in natural bin order, handed over in the transform's order
    y = (rng.standard_normal((batch, n_pol, n)) + 1j * rng.standard_normal((batch, n_pol, n)))
    y = y.astype(np.complex64)
    plan = ssfm.Plan(link(n_pol, n))
    try:
        info = plan.info
        order = storage_of_bins(info, n, np.arange(n))  # position of bin k
        held = np.empty_like(y)
        held[..., order] = y
        t = torch.from_numpy(held).cuda()
        ssfm.ssfm_dft(plan.handle, t, inverse=True)
        torch.cuda.synchronize()
        got = t.cpu().numpy().astype(np.complex128)
    finally:
        plan.close()
    times = sampled_bins(rng, n)
    for b in sorted({0, batch - 1}):
        want = oracle.dft_bins(y[b].astype(np.complex128), times, inverse=True)
        check(got[b][:, times], want, 1e-6, what=f"realisation {b}")


@pytest.mark.parametrize("n,n_pol", [(2048, 2), (1 << 16, 2)])
@pytest.mark.parametrize("arithmetic", ["fp64", "fp32"])
def test_round_trip_returns_n_times_the_input(ssfm, n, n_pol, arithmetic):
    rng = np.random.default_rng(n)
    x = (rng.standard_normal((4, n_pol, n)) + 1j * rng.standard_normal((4, n_pol, n)))
    x = x.astype(np.complex64)
    plan = ssfm.Plan(link(n_pol, n), arithmetic=arithmetic)
    try:
        t = torch.from_numpy(x).cuda()
        ssfm.ssfm_dft(plan.handle, t, inverse=False)
        ssfm.ssfm_dft(plan.handle, t, inverse=True)
        torch.cuda.synchronize()
        got = t.cpu().numpy().astype(np.complex128)
    finally:
        plan.close()
    # FP64 transforms: complex64 storage between them; FP32: ~u log2(n)
    check(got, n * x.astype(np.complex128), 1e-6 if arithmetic == "fp64" else 2e-6)


def test_dft_rejects_bad_direction(ssfm):
    plan = ssfm.Plan(link(1, 4096))
    try:
        t = torch.zeros((1, 1, 4096), dtype=torch.complex64, device="cuda")
        lib = ssfm.load_library()
        import ctypes
        rc = lib.ssfm_dft(plan.handle, ctypes.c_void_p(t.data_ptr()), 1, 2, None)
        assert rc == ssfm.SSFM_EINVAL
    finally:
        plan.close()
