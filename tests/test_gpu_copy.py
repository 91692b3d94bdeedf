"""The measurement utilities: ssfm_stream_copy, the bandwidth reference (an
exact copy, rejection of misaligned buffers and sizes), and
ssfm_orchestration_probe (every method completes with a positive time; bad
arguments rejected before any device work)."""

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


@pytest.mark.parametrize("method", [0, 1, 2])
@pytest.mark.parametrize("workgroups", [1, 64, 256])
def test_orchestration_probe_runs(ssfm, method, workgroups):
    print(f"case method={method} workgroups={workgroups}", flush=True)
    us = ssfm.ssfm_orchestration_probe(method, workgroups, 50)
    assert 0.0 < us < 1e4


def test_orchestration_probe_rejects_bad_arguments(ssfm):
    import ctypes
    lib = ssfm.load_library()
    us = ctypes.c_double(0.0)
    assert lib.ssfm_orchestration_probe(3, 8, 10, None, ctypes.byref(us)) == ssfm.SSFM_EINVAL
    assert lib.ssfm_orchestration_probe(0, 0, 10, None, ctypes.byref(us)) == ssfm.SSFM_EINVAL
    assert lib.ssfm_orchestration_probe(0, 8, 0, None, ctypes.byref(us)) == ssfm.SSFM_EINVAL
    assert lib.ssfm_orchestration_probe(0, 8, 1 << 20, None, ctypes.byref(us)) == ssfm.SSFM_EINVAL
    # more workgroups than can be resident at once
    assert lib.ssfm_orchestration_probe(2, 1 << 16, 10, None, ctypes.byref(us)) == ssfm.SSFM_EINVAL
    assert lib.ssfm_orchestration_probe(0, 8, 10, None, None) == ssfm.SSFM_EINVAL
