"""The read-rate diagnostic (gkl_read_rate): a plain streaming read of a device
buffer, the practical ceiling the product kernels are compared with."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_1808_03374_amd as m
    return m


def test_read_rate_times_a_read(gk):
    buf = torch.zeros(256 << 20, dtype=torch.uint8, device="cuda")
    ms = gk.gkl_read_rate(buf, reps=3)
    gbps = buf.numel() / (ms * 1e-3) / 1e9
    # a 256 MB read: well above PCIe rates and below the 8 TB/s HBM peak
    assert 100.0 < gbps < 8000.0
    # a ragged length (the tail past a multiple of 16 bytes is not read)
    assert gk.gkl_read_rate(buf[: (1 << 20) + 7], reps=1) > 0.0


def test_read_rate_rejects_bad_arguments(gk):
    buf = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    for bad in (buf[1:], buf[:8]):          # misaligned, shorter than 16 bytes
        with pytest.raises(gk.GKLError) as e:
            gk.gkl_read_rate(bad, reps=1)
        assert e.value.status == gk.GKL_ERR_INVALID
    with pytest.raises(gk.GKLError):
        gk.gkl_read_rate(buf, reps=0)
