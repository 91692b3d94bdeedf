"""ssfm_adjoint_noalloc (the adjoint with the library's fixed device scratch,
no allocation) against ssfm_adjoint, the entry point that allocates its
workspace: the same kernels in the same order, so the results must agree bit
for bit; both are also held to the FP64 oracle's adjoint."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from fieldcheck import check
from workloads import Link, dual_pol_field

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 128 << 20


@pytest.fixture(scope="module")
def ssfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_03509_amd as m
    m.load_library()
    return m


def link(n, spans, steps):
    return Link(n_pol=2, n_samples=n, sample_rate_hz=128e9, span_km=80.0, n_spans=spans,
                steps_per_span=steps, alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7,
                gamma_per_w_km=1.3, edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True)


def test_noalloc_adjoint_equals_adjoint(ssfm):
    n, spans, steps = 1 << 16, 3, 4
    ln = link(n, spans, steps)
    per_real = (spans + 2) * 2 * n * 8
    b_max = SCRATCH_BYTES // per_real
    plan = ssfm.Plan(ln)
    try:
        # the largest batch the scratch holds, then a smaller one: the second
        # call reuses what the first left in the scratch
        for b, seed in ((b_max, 11), (3, 12)):
            print(f"case n={n} spans={spans} batch={b} seed={seed}", flush=True)
            rng = np.random.default_rng(b)
            x = np.stack([dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 6.0) for _ in range(b)])
            g = np.stack([dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 0.0) for _ in range(b)])
            xt = torch.from_numpy(x.astype(np.complex64)).cuda()
            gt = torch.from_numpy(g.astype(np.complex64)).cuda()
            ref = gt.clone()
            plan.adjoint(xt, ref, seed=seed)
            out = gt.clone()
            ssfm.ssfm_adjoint_noalloc(plan.handle, xt, out, seed=seed)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), f"batch {b}: differs from ssfm_adjoint"
            got = out.cpu().numpy().astype(np.complex128)
            for r in (0, b - 1):
                want = oracle.adjoint(x[r], g[r], ln, seed=seed, realization=r)
                check(got[r], want, 1e-5, what=f"batch {b} realisation {r}")
    finally:
        plan.close()


def test_noalloc_adjoint_lds_path_equals_adjoint(ssfm):
    # the LDS-resident path (one launch per call): two calls, the second
    # with a smaller batch, bit for bit against ssfm_adjoint
    n, spans, steps = 4096, 2, 3
    ln = link(n, spans, steps)
    plan = ssfm.Plan(ln)
    try:
        for b, seed in ((6, 21), (2, 22)):
            print(f"case n={n} spans={spans} batch={b} seed={seed}", flush=True)
            rng = np.random.default_rng(100 + b)
            x = np.stack([dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 6.0) for _ in range(b)])
            g = np.stack([dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 0.0) for _ in range(b)])
            xt = torch.from_numpy(x.astype(np.complex64)).cuda()
            gt = torch.from_numpy(g.astype(np.complex64)).cuda()
            ref = gt.clone()
            plan.adjoint(xt, ref, seed=seed)
            out = gt.clone()
            ssfm.ssfm_adjoint_noalloc(plan.handle, xt, out, seed=seed)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), f"batch {b}: differs from ssfm_adjoint"
            got = out.cpu().numpy().astype(np.complex128)
            want = oracle.adjoint(x[b - 1], g[b - 1], ln, seed=seed, realization=b - 1)
            check(got[b - 1], want, 1e-5, what=f"batch {b}")
    finally:
        plan.close()


def test_noalloc_adjoint_rejects_oversized(ssfm):
    n, spans = 1 << 16, 3
    ln = link(n, spans, 2)
    b = SCRATCH_BYTES // ((spans + 2) * 2 * n * 8) + 1
    plan = ssfm.Plan(ln)
    try:
        x = torch.zeros((b, 2, n), dtype=torch.complex64, device="cuda")
        g = torch.zeros_like(x)
        with pytest.raises(ssfm.SsfmError) as e:
            ssfm.ssfm_adjoint_noalloc(plan.handle, x, g, seed=1)
        assert e.value.status == ssfm.SSFM_EINVAL
        assert "scratch" in str(e.value)
    finally:
        plan.close()
