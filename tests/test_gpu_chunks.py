"""Batches above the plan's chunk size run as sequential chunks, each as one
or more concurrent parts: the forward call (direct and graph replay) and the
adjoint give the bits of one pass over the whole batch, and the oracle's
result.  SSFM_CHUNK_MIB, read when a plan
is built, sets the chunk size (0: none), so small fields exercise several
chunks, including a shorter last one."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from fieldcheck import check
from workloads import Link, dual_pol_field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_03509_amd as m
    m.load_library()
    return m


def link(n_pol, n):
    return Link(n_pol=n_pol, n_samples=n, sample_rate_hz=128e9, span_km=80.0, n_spans=2,
                steps_per_span=3, alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7,
                gamma_per_w_km=1.3, edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True)


def plan_with_chunks(ssfm, monkeypatch, ln, mib):
    monkeypatch.setenv("SSFM_CHUNK_MIB", str(mib))
    plan = ssfm.Plan(ln)
    monkeypatch.delenv("SSFM_CHUNK_MIB")
    return plan


# (n, n_pol, batch): 2^14 dual-pol is 256 KiB per realisation, so 1 MiB
# chunks hold 4 realisations (the adjoint's, two fields each, 2); 2^16
# single-pol is 512 KiB (chunks of 2 and 1)
# parts: each chunk of the chunked plan as that many concurrent parts (the
# one-pass plan runs on one stream)
@pytest.mark.parametrize("n,n_pol,batch,parts", [(1 << 14, 2, 7, 1), (1 << 16, 1, 5, 1),
                                                 (1 << 14, 2, 7, 2), (1 << 16, 1, 5, 2)])
def test_chunked_calls_equal_one_pass(ssfm, monkeypatch, n, n_pol, batch, parts):
    print(f"case n={n} n_pol={n_pol} batch={batch} parts={parts}", flush=True)
    ln = link(n_pol, n)
    rng = np.random.default_rng(n + batch)
    x = np.stack([dual_pol_field(rng, n_pol, n, 2, 64e9, 0.1, 4.0) for _ in range(batch)])
    g = np.stack([dual_pol_field(rng, n_pol, n, 2, 64e9, 0.1, 0.0) for _ in range(batch)])
    x = x.astype(np.complex64)
    g = g.astype(np.complex64)
    whole = plan_with_chunks(ssfm, monkeypatch, ln, 0)
    chunked = plan_with_chunks(ssfm, monkeypatch, ln, 1)
    whole.set_forward_streams(1)
    chunked.set_forward_streams(parts)
    try:
        assert whole.info["chunk_realisations"] == 0
        per = n_pol * n * 8
        assert chunked.info["chunk_realisations"] == (1 << 20) // per
        # forward: direct, then the captured and replayed repeats
        ref = torch.from_numpy(x).cuda()
        whole.forward(ref, seed=17)
        outs = []
        for _ in range(3):
            t = torch.from_numpy(x).cuda()
            chunked.forward(t, seed=17)
            outs.append(t)
        torch.cuda.synchronize()
        for t in outs:
            assert torch.equal(t, ref)
        got = ref.cpu().numpy().astype(np.complex128)
        for b in (0, batch - 1):
            check(got[b], oracle.propagate(x[b], ln, seed=17, realization=b), 2e-6,
                  what=f"realisation {b}")
        # adjoint, span checkpoints and in-span rebuild
        xa = torch.from_numpy(x).cuda()
        ga = torch.from_numpy(g).cuda()
        whole.adjoint(xa, ga, seed=17)
        gb = torch.from_numpy(g).cuda()
        chunked.adjoint(xa, gb, seed=17)
        torch.cuda.synchronize()
        assert torch.equal(ga, gb)
        got = gb.cpu().numpy().astype(np.complex128)
        b = batch - 1
        want = oracle.adjoint(x[b], g[b], ln, seed=17, realization=b)
        check(got[b], want, 1e-5, what=f"adjoint realisation {b}")
    finally:
        whole.close()
        chunked.close()
