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


def test_network_gain_at_equal_budget():
    """The same reduced budget (the learned run's particles and iterations),
    batched, with and without the network: centring and scaling the template
    by the trained network tracks far better than carrying the previous
    frame's state (8 held-out sequences, 40 frames)."""
    from paper_2105_05600_amd import rose, train_proposal as tp
    import synth
    with open(os.path.splitext(WEIGHTS)[0] + ".json") as f:
        meta = json.load(f)
    n, frames = 8, 40
    seqs = [tp.make_sequence(55000 + 10 * i, frames, 320, 240) for i in range(n)]
    depths = [[torch.from_numpy(d).cuda() for d in sq.depths(range(frames), workers=16)] for sq in seqs]
    net = rose.Mlp(tp.FEATURE_DIM, 256, 12, max_batch=64)
    P = net.pack(tp.load(WEIGHTS))
    iters = meta.get("iters", 0) or 20
    pst_small = rose.pst_sample(meta.get("particles", 4096), 5600)
    pst_plain = rose.pst_sample(10240, 5600)
    plain = rose.track_params(max_iters=20, stride=4)
    small = rose.track_params(max_iters=iters, stride=4)
    lp = rose.learned_params(scale=8, kappa=meta["kappa"], delta=meta["delta"], iters=iters)

    def run(learned):
        vols, states = [], (rose.TrackState * n)()
        for i, sq in enumerate(seqs):
            vol = rose.Tsdf(sq.dims, sq.vox, sq.mu, sq.origin)
            vol.integrate(depths[i][0], sq.K, sq.poses[0].q, sq.poses[0].t)
            vols.append(vol)
            states[i] = rose.track_state(sq.poses[0].q, sq.poses[0].t, [0.55] * 6)
        b = rose.Batch(vols, [sq.K for sq in seqs], [pst_small] * n, [small] * n, use_graph=False)
        work = torch.zeros(n * (tp.LOW_W * tp.LOW_H + tp.FEATURE_DIM + 12), device="cuda")
        est = [[np.array(sq.poses[0].t)] for sq in seqs]
        vel = [[0.0] * 6 for _ in range(n)]
        for f in range(1, frames):
            prev = [(list(states[i].pose.q), list(states[i].pose.t)) for i in range(n)]
            if learned:
                rose.batch_track_learned(b, [d[f] for d in depths], net, P, work, vel, lp, [pst_plain] * n,
                                         [plain] * n, states)
            else:
                b.track([d[f] for d in depths], states)
            for i, sq in enumerate(seqs):
                q, t = list(states[i].pose.q), list(states[i].pose.t)
                vel[i] = rose.chart_log(prev[i][0], prev[i][1], q, t)
                est[i].append(np.array(t))
                vols[i].integrate(depths[i][f], sq.K, q, t)
        b.close()
        for v in vols:
            v.close()
        return [synth.ate(np.array(e), np.array([p.t for p in sq.poses[:frames]]))[1] for e, sq in zip(est, seqs)]

    with_net = run(True)
    without = run(False)
    print(f"mean ATE with the network {np.mean(with_net):.4f} m, without {np.mean(without):.4f} m; "
          f"medians {np.median(with_net):.4f} / {np.median(without):.4f} m")
    assert np.mean(with_net) < np.mean(without)
    assert np.median(with_net) < np.median(without)
