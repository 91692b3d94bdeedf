"""ssfm_plan_autotune: the measured launch shape is recorded per batch and
does not change results (every variant computes each transform with the same
FP64 arithmetic), bit for bit, including through graph replay."""

import numpy as np
import pytest

from workloads import Link, dual_pol_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ssfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_03509_amd as mod
    mod.load_library()
    return mod


LINK = Link(n_pol=2, n_samples=1 << 16, sample_rate_hz=128e9, span_km=80.0, n_spans=1,
            steps_per_span=6, alpha_db_per_km=0.2, beta2_ps2_per_km=-21.7,
            gamma_per_w_km=1.3, edfa_gain_db=16.0, edfa_nf_db=5.0, ase=True)


@pytest.mark.parametrize("batch", [1, 6, 64])
def test_tuned_shape_gives_identical_results(ssfm, batch):
    print(f"autotune batch={batch}", flush=True)
    rng = np.random.default_rng(batch)
    a0 = np.stack([dual_pol_field(rng, 2, LINK.n_samples, 2, 64e9, 0.1, 2.0)
                   for _ in range(batch)]).astype(np.complex64)
    x = torch.from_numpy(a0).cuda()
    ref_plan = ssfm.Plan(LINK, device=0)
    ref = x.clone()
    ref_plan.forward(ref, seed=3)
    plan = ssfm.Plan(LINK, device=0)
    info = plan.autotune(batch)
    print(f"  chose columns={info['columns']} rows={info['row_lanes']} us={info['us_per_step']}",
          flush=True)
    assert info["columns"] in (2, 4, 8)
    assert info["row_lanes"] in (64, 256)
    assert len(info["us_per_step"]) == 4 and all(t > 0 for t in info["us_per_step"])
    for _ in range(3):  # direct, capture, replay
        y = x.clone()
        plan.forward(y, seed=3)
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
    ref_plan.close()
    plan.close()


def test_lds_path_has_nothing_to_tune(ssfm):
    plan = ssfm.Plan(LINK.replace(n_samples=4096), device=0)
    info = plan.autotune(8)
    assert info["columns"] == 0 and info["row_lanes"] == 0 and info["us_per_step"] == []
    plan.close()
