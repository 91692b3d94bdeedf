"""Failure paths of the C ABI on the GPU: an allocation that fails while a
plan builds its tables returns SSFM_ENOMEM and leaves no device memory
behind (fault injection: SSFM_FAIL_ALLOC=k makes the plan's k-th table
allocation fail)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import Link

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_03509_amd as m
    m.load_library()
    return m


def link(n):
    return Link(n_pol=2, n_samples=n, sample_rate_hz=128e9, span_km=80.0, n_spans=2,
                steps_per_span=4, alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7,
                gamma_per_w_km=1.3, edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True)


# tables: H half, H full, kappa, then the twiddles (one table on the
# LDS-resident path, four on the four-step path)
@pytest.mark.parametrize("n,tables", [(4096, 4), (1 << 18, 7)])
def test_plan_allocation_failure_returns_enomem_without_leak(ssfm, monkeypatch, n, tables):
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for k in range(1, tables + 1):
        monkeypatch.setenv("SSFM_FAIL_ALLOC", str(k))
        for _ in range(40 if k == tables else 1):
            with pytest.raises(ssfm.SsfmError) as ei:
                ssfm.ssfm_plan(link(n), 0)
            assert ei.value.status == ssfm.SSFM_ENOMEM
            assert "SSFM_FAIL_ALLOC" in str(ei.value)
    # one past the last table: nothing fails
    monkeypatch.setenv("SSFM_FAIL_ALLOC", str(tables + 1))
    h = ssfm.ssfm_plan(link(n), 0)
    ssfm.ssfm_plan_destroy(h)
    monkeypatch.delenv("SSFM_FAIL_ALLOC")
    torch.cuda.synchronize()
    # 40 failed plans at 2^18 would leave 40 x 8 MiB of dispersion tables
    # behind if the earlier tables leaked
    assert abs(torch.cuda.mem_get_info()[0] - free0) < 64 << 20
