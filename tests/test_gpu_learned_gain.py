"""What the trained proposal network gains (committed weights, trained on the
GPU by the library's own BF16 kernels), on 32 held-out fast-motion sequences
(320x240, 1-4 m/s, seeds 56000+: never used for training, for choosing kappa
and delta or for any earlier comparison), 40 frames each, every run fused at
its own tracked poses:

* plain PST (10240 particles, 20 iterations) one sequence after another
  (the single-sequence path in the switching mode), and the same budget
  batched in the switching mode (a control for the batching alone: its
  poses equal the single path's bit for bit, so only its speed differs);
* the learned proposal batched (pso_batch_track_learned: the network's
  centre and axis lengths, the small template and iteration count, plain
  PST as per-sequence fallback), with the trained network and with an
  untrained network of the same shape under the same fallback rule (equal
  budget, equal fallback: the difference is the network).

Asserted: (i) the trained network tracks better than the untrained one
(mean and median ATE); (ii) learned + batched runs more frames/s than plain
PST one sequence after another at equal or better mean and median ATE;
(iii) it is also faster than plain PST batched, so the gain is not the
batching alone.  Printed: every mode's frames/s, ATE and fallbacks."""
import json

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_learned_batched_gain_on_32_sequences():
    assert torch.cuda.is_available()
    from paper_2105_05600_amd import bench_batch
    res = bench_batch.learned_comparison(32, 40, 56000, modes=("plain_single", "plain_batched", "learned",
                                                                "untrained"),
                                         log=lambda m: print(m, flush=True))
    print(json.dumps({m: {k: v for k, v in r.items() if k != "ate_rmse_m"} for m, r in res.items()}, indent=1))
    ps, pb, ln, un = res["plain_single"], res["plain_batched"], res["learned"], res["untrained"]
    # the batching control changes no pose
    assert np.array_equal(ps["ate_rmse_m"], pb["ate_rmse_m"])
    # (i) trained beats untrained at equal budget and fallback rule
    assert ln["ate_rmse_mean_m"] < un["ate_rmse_mean_m"]
    assert ln["ate_rmse_median_m"] < un["ate_rmse_median_m"]
    # (ii) learned + batched beats plain PST on frames/s at <= mean and median ATE
    assert ln["frames_per_s"] > ps["frames_per_s"]
    assert ln["ate_rmse_mean_m"] <= ps["ate_rmse_mean_m"]
    assert ln["ate_rmse_median_m"] <= ps["ate_rmse_median_m"]
    # (iii) and is faster than plain PST batched
    assert ln["frames_per_s"] > pb["frames_per_s"]
