"""The measured HBM read rate the memory-bound kernels are reported against
(stwr_ctx_read_rate): a plain streaming read of a device buffer too large for
the caches.  Checked: the rate is positive and below the device's published
8 TB/s HBM peak (a rate above it would mean the caches served the buffer);
the buffer is left as it was; sizes under 64 MiB or not a multiple of 16
bytes are refused with STWR_ERR_ARG."""
import pytest

from gpu_common import ctx, log, torch_cuda

pytestmark = pytest.mark.gpu

HBM_PEAK_GBS = 8000.0


def test_read_rate_is_a_plausible_hbm_rate():
    torch = torch_cuda()
    buf = torch.arange(1 << 29, dtype=torch.float32, device="cuda")   # 2 GiB
    before = buf[::4097].clone()
    gbs = ctx().read_rate(buf, 3)
    log(f"measured read rate {gbs:.1f} GB/s")
    assert 500.0 < gbs < 1.02 * HBM_PEAK_GBS
    assert torch.equal(buf[::4097], before)


def test_read_rate_rejects_bad_sizes():
    torch = torch_cuda()
    from paper_2407_13997_amd import binding
    small = torch.zeros(1 << 20, dtype=torch.float32, device="cuda")   # 4 MiB
    with pytest.raises(binding.StwrError) as e:
        ctx().read_rate(small, 1)
    assert e.value.code == -1   # STWR_ERR_ARG
    odd = torch.zeros((64 << 20) + 4, dtype=torch.uint8, device="cuda")
    with pytest.raises(binding.StwrError) as e:
        ctx().read_rate(odd, 1)
    assert e.value.code == -1   # STWR_ERR_ARG
