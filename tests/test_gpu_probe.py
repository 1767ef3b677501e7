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
