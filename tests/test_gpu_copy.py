"""ssfm_stream_copy, the bandwidth reference of the measurements: an exact
copy, rejection of misaligned buffers and sizes."""

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ssfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_03509_amd as mod
    mod.load_library()
    return mod


@pytest.mark.parametrize("elems", [2, 1000, 1 << 20, (1 << 22) + 6])
def test_copy_is_exact(ssfm, elems):
    src = torch.randn(elems, dtype=torch.complex64, device="cuda")
    dst = torch.zeros_like(src)
    ssfm.ssfm_stream_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


def test_copy_rejects_bad_arguments(ssfm):
    lib = ssfm.load_library()
    a = torch.zeros(64, dtype=torch.complex64, device="cuda")
    b = torch.zeros(64, dtype=torch.complex64, device="cuda")
    assert lib.ssfm_stream_copy(a.data_ptr() + 8, b.data_ptr(), 256, None) == ssfm.SSFM_EINVAL
    assert lib.ssfm_stream_copy(a.data_ptr(), b.data_ptr(), 24, None) == ssfm.SSFM_EINVAL
    assert lib.ssfm_stream_copy(None, b.data_ptr(), 256, None) == ssfm.SSFM_EINVAL
    assert lib.ssfm_stream_copy(a.data_ptr(), b.data_ptr(), 0, None) == ssfm.SSFM_OK
