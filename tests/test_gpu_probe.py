"""The gather-rate probe (the fitness kernel's gather roofline) runs and
reports a plausible rate: every load is counted, an L2-resident region is
served faster than one far larger than the L2, and the sink is untouched."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_gather_probe_rates():
    from paper_2105_05600_amd import rose
    rates = {}
    for mib in (2, 256):
        lines = mib * (1 << 20) // 128
        buf = torch.rand(8 * lines * 32, device="cuda")
        sink = torch.zeros(512, device="cuda")
        n = rose.gather_peak(buf, lines, 512, 16, sink)
        assert n == 512 * 256 * 16 * 8
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rose.gather_peak(buf, lines, 512, 16, sink)
        e1.record()
        torch.cuda.synchronize()
        rates[mib] = n / (e0.elapsed_time(e1) * 1e-3)
        assert torch.count_nonzero(sink) == 0
    print(rates)
    assert rates[2] > 1e10 and rates[2] > rates[256]


def test_l2_read_probe_rate():
    """The L2 -> CU read probe over an L2-resident region (2 MiB per XCD):
    every byte is counted, the rate is plausible (above the HBM peak's order,
    below 100 TB/s) and the sink is untouched."""
    from paper_2105_05600_amd import rose
    region = 2 * (1 << 20) // 16
    buf = torch.rand(8 * region * 4, device="cuda")
    sink = torch.zeros(2048, device="cuda")
    rose.l2_read_peak(buf, region, 2048, 1, sink)  # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    n = rose.l2_read_peak(buf, region, 2048, 2, sink)
    e1.record()
    torch.cuda.synchronize()
    assert n == 2048 * 2 * region * 16
    rate = n / (e0.elapsed_time(e1) * 1e-3)
    print(f"L2 -> CU reads: {rate / 1e12:.2f} TB/s")
    assert torch.count_nonzero(sink) == 0
    assert 2e12 < rate < 1e14
