"""The batched learned frame step (pso_batch_track_learned: raycasts and
features per sequence, one network forward over all sequences, one batched
small-template step, per-sequence plain fallback) equals the single learned
frame (pso_track_frame_learned) sequence by sequence, frame after frame:
poses, axis lengths, fitness and fallback decisions bit for bit; with the
fixed launch shape (4, 2) and in the switching mode, where every sequence
here (over 2^23 evaluations per iteration) takes the single path's own
fitness launches inside the batch."""
import json
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2105_05600_amd",
                       "weights", "proposal.npz")


@pytest.mark.parametrize("shape", [(4, 2), (0, 0)])
@pytest.mark.parametrize("always_fall_back", [False, True])
def test_batch_learned_equals_single(always_fall_back, shape):
    from paper_2105_05600_amd import rose
    rose.set_fitness_shape(*shape)
    try:
        _batch_learned_equals_single(rose, always_fall_back)
    finally:
        rose.set_fitness_shape(4, 2)


def _batch_learned_equals_single(rose, always_fall_back):
    from paper_2105_05600_amd import train_proposal as tp
    with open(os.path.splitext(WEIGHTS)[0] + ".json") as f:
        meta = json.load(f)
    n_seq, n_frames = 4, 8
    seqs = [tp.make_sequence(51000 + 10 * i, n_frames, 320, 240) for i in range(n_seq)]
    depths = [[torch.from_numpy(d).cuda() for d in sq.depths(range(n_frames), workers=16)] for sq in seqs]
    net = rose.Mlp(tp.FEATURE_DIM, 256, 12, max_batch=64)
    P = net.pack(tp.load(WEIGHTS))
    n_small, iters = meta.get("particles", 4096), meta.get("iters", 0) or 20
    pst_small = rose.pst_sample(n_small, 5600)
    pst_plain = rose.pst_sample(10240, 5600)
    # delta = -1: every learned run "regresses", so every frame takes the
    # plain fallback (which reallocates the handles' scratch under the batch)
    delta = -1.0 if always_fall_back else meta["delta"]
    lp = rose.learned_params(scale=8, kappa=meta["kappa"], delta=delta, iters=iters)
    plain = rose.track_params(max_iters=20, stride=4)
    small = rose.track_params(max_iters=iters, stride=4)

    def start(i):
        sq = seqs[i]
        vol = rose.Tsdf(sq.dims, sq.vox, sq.mu, sq.origin)
        st = rose.track_state(sq.poses[0].q, sq.poses[0].t, [1.0] * 6, tsdf_built=False)
        rose.track_frame(vol, depths[i][0], sq.K, pst_plain, plain, st)
        vol.integrate(depths[i][0], sq.K, sq.poses[0].q, sq.poses[0].t)
        st.tsdf_built = 1
        return vol, st

    # single learned frames
    ref = []
    work1 = torch.zeros(tp.LOW_W * tp.LOW_H + tp.FEATURE_DIM + 12, device="cuda")
    for i, sq in enumerate(seqs):
        vol, st = start(i)
        vel = [0.0] * 6
        rows = []
        for f in range(1, n_frames):
            q0, t0 = list(st.pose.q), list(st.pose.t)
            r = rose.track_frame_learned(vol, depths[i][f], sq.K, pst_small, pst_plain, net, P, work1, vel, plain,
                                         lp, st)
            rows.append((list(st.pose.q), list(st.pose.t), list(st.r), st.rho, r["fallback"]))
            vel = rose.chart_log(q0, t0, list(st.pose.q), list(st.pose.t))
            vol.integrate(depths[i][f], sq.K, st.pose.q, st.pose.t)
        ref.append(rows)
        vol.close()

    # batched learned frames
    vols, sts = zip(*[start(i) for i in range(n_seq)])
    states = (rose.TrackState * n_seq)(*sts)
    b = rose.Batch(list(vols), [sq.K for sq in seqs], [pst_small] * n_seq, [small] * n_seq, use_graph=False)
    work = torch.zeros(n_seq * (tp.LOW_W * tp.LOW_H + tp.FEATURE_DIM + 12), device="cuda")
    vel = [[0.0] * 6 for _ in range(n_seq)]
    fallbacks = 0
    for f in range(1, n_frames):
        prev = [(list(states[i].pose.q), list(states[i].pose.t)) for i in range(n_seq)]
        res = rose.batch_track_learned(b, [d[f] for d in depths], net, P, work, vel, lp, [pst_plain] * n_seq,
                                       [plain] * n_seq, states)
        for i, sq in enumerate(seqs):
            q, t, r1, rho, fb = ref[i][f - 1]
            assert list(states[i].pose.q) == q and list(states[i].pose.t) == t, (i, f)
            assert list(states[i].r) == r1 and states[i].rho == rho and res[i]["fallback"] == fb, (i, f)
            fallbacks += int(fb)
            vel[i] = rose.chart_log(prev[i][0], prev[i][1], list(states[i].pose.q), list(states[i].pose.t))
            vols[i].integrate(depths[i][f], sq.K, states[i].pose.q, states[i].pose.t)
    print(f"{n_seq} sequences x {n_frames - 1} frames, {fallbacks} fallbacks")
    if always_fall_back:
        assert fallbacks == n_seq * (n_frames - 1)
    b.close()
    for v in vols:
        v.close()
