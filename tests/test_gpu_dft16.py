"""Radix-16 DFT stage prototype (ssfm_dft16_rounds): the FFTs' vector
butterfly and the matrix-core product against the direct-DFT oracle."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_03509_amd as m
    m.load_library()
    return m


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("count,rounds", [(64, 1), (64, 3), (1024, 5), (192, 0)])
def test_dft16_rounds_match_oracle(ssfm, method, count, rounds):
    print(f"case method={method} count={count} rounds={rounds}", flush=True)
    rng = np.random.default_rng(count + rounds)
    x = rng.standard_normal((count, 16)) + 1j * rng.standard_normal((count, 16))
    t = torch.from_numpy(x).cuda()
    ssfm.ssfm_dft16_rounds(method, t, rounds)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    want = oracle.dft16_rounds(x, rounds)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    assert err < 1e-14, err


def test_dft16_methods_agree_and_reject_bad_calls(ssfm):
    rng = np.random.default_rng(9)
    x = rng.standard_normal((128, 16)) + 1j * rng.standard_normal((128, 16))
    a = torch.from_numpy(x).cuda()
    b = a.clone()
    ssfm.ssfm_dft16_rounds(0, a, 8)
    ssfm.ssfm_dft16_rounds(1, b, 8)
    torch.cuda.synchronize()
    assert np.allclose(a.cpu().numpy(), b.cpu().numpy(), rtol=0, atol=1e-13)
    bad = torch.zeros((100, 16), dtype=torch.complex128, device="cuda")
    with pytest.raises(ssfm.SsfmError):
        ssfm.ssfm_dft16_rounds(0, bad, 1)      # count not a multiple of 64
    with pytest.raises(ssfm.SsfmError):
        ssfm.ssfm_dft16_rounds(2, a, 1)        # no such method
    with pytest.raises(ssfm.SsfmError):
        ssfm.ssfm_dft16_rounds(0, a, -1)       # negative rounds
