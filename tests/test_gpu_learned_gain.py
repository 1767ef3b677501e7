"""What the trained proposal network gains (committed weights, trained on the
GPU by the library's own BF16 kernels): on held-out fast-motion sequences
(320x240, 1-4 m/s, seeds never used for training or for choosing kappa and
delta) the learned frame -- 4096 particles centred and scaled by the network,
plain 10240-particle PST as fallback -- is compared with plain PST and with the
same path driven by an untrained network of the same shape.

Asserted: the learned frame is at least 1.3x faster than plain PST (it
evaluates 2.5x fewer particle-point pairs) and does not diverge (mean ATE
within 3x plain PST's + 5 cm).  Printed beside it: the ATE of all three.  On
these sequences plain PST keeps the lower mean ATE (the proposal trades
accuracy for speed), and the untrained network -- whose output leaves the
previous pose as centre with the maximum scale -- tracks about as well as the
trained one."""
import json
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2105_05600_amd",
                       "weights", "proposal.npz")


def test_trained_proposal_gain():
    assert torch.cuda.is_available()
    from paper_2105_05600_amd import rose, train_proposal as tp
    import synth.mlp_init as mlp_init
    with open(os.path.splitext(WEIGHTS)[0] + ".json") as f:
        meta = json.load(f)
    net = rose.Mlp(tp.FEATURE_DIM, 256, 12, max_batch=512)
    P = net.pack(tp.load(WEIGHTS))
    untrained = net.pack(mlp_init.init_params(1))
    seeds = [50000, 50010, 50020]
    rows = tp.evaluate(net, P, seeds, 90, 320, 240, n_small=meta.get("particles", 4096), workers=16,
                       kappa=meta["kappa"], delta=meta["delta"], modes=("plain", "learned", "untrained"),
                       nets={"untrained": untrained}, learned_iters=meta.get("iters", 0))
    s = tp.summarize(rows, ("plain", "learned", "untrained"))
    print(json.dumps(s, indent=1))
    assert s["learned"]["frames_per_s_mean"] >= 1.3 * s["plain"]["frames_per_s_mean"]
    assert s["learned"]["ate_rmse_mean_m"] <= 3.0 * s["plain"]["ate_rmse_mean_m"] + 0.05
    assert all(np.isfinite(r["learned"]["ate_rmse_m"]) for r in rows)
