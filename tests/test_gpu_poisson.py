"""6D Poisson-disk template on the GPU equals the oracle's bit for bit
(integer-exact dart throwing over the same candidate stream): rows, rows
accepted and candidates drawn, including r_min = 0 (the i.i.d. template), a
budget that runs out, and a full-size 10240-row template."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,seed,r,budget", [(1, 1, 0.3, 100), (777, 5600, 0.0, 1000), (300, 3, 0.35, 200000),
                                             (1024, 5600, 0.3, 200000), (1000, 9, 0.45, 500),
                                             (600, 11, 0.3, 0), (10240, 5600, 0.2392, 100000)])
def test_poisson_bit_exact(orc, n, seed, r, budget):
    from paper_2105_05600_amd import rose
    g, got_g, drawn_g = rose.pst_poisson(n, seed, r, budget)
    o, got_o, drawn_o = orc.pst_poisson(n, seed, r, budget)
    torch.cuda.synchronize()
    assert (got_g, drawn_g) == (got_o, drawn_o)
    assert np.array_equal(g.cpu().numpy().view(np.uint32), o.view(np.uint32))
    if r == 0.0:
        iid, _ = orc.pst_sample(n, seed)
        assert np.array_equal(o, iid)
