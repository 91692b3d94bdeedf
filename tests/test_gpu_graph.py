"""Launch-sequence replay: a repeated ssfm_forward call replays a captured
graph.  Every replay, with eager work and synchronisations in between, must
equal the direct-launch result bit for bit."""

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import Link, dual_pol_field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_03509_amd as m
    m.load_library()
    return m


def test_graph_replays_equal_direct_launches(ssfm, monkeypatch):
    n = 1 << 15
    ln = Link(n_pol=2, n_samples=n, sample_rate_hz=128e9, span_km=80.0, n_spans=2,
              steps_per_span=4, alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7,
              gamma_per_w_km=1.3, edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True)
    rng = np.random.default_rng(2)
    xs = [torch.from_numpy(dual_pol_field(rng, 2, n, 2, 64e9, 0.1, 3.0).astype(np.complex64))
          [None].cuda() for _ in range(3)]
    plan = ssfm.Plan(ln)
    monkeypatch.setenv("SSFM_GRAPH", "0")
    direct = []
    for x in xs:
        y = x.clone()
        plan.forward(y, seed=9)
        direct.append(y)
    torch.cuda.synchronize()
    monkeypatch.delenv("SSFM_GRAPH")
    t = torch.empty_like(xs[0])
    for rep in range(7):
        k = rep % 3
        t.copy_(xs[k])                      # eager work between replays
        scratch = (xs[(k + 1) % 3] * 2).sum()
        plan.forward(t, seed=9)             # rep 0 direct, 1 capture, then replays
        torch.cuda.synchronize()
        assert torch.equal(t, direct[k]), f"replay {rep} differs"
        assert torch.isfinite(scratch.real)
    # another seed: a new key, run directly and again correct
    y = xs[0].clone()
    plan.forward(y, seed=10)
    t.copy_(xs[0])
    plan.forward(t, seed=10)
    torch.cuda.synchronize()
    assert torch.equal(t, y)
    plan.close()
