"""The batched tracker at the uneven sizes of the many-sequence workload:
volumes 256^3 / 384^3 / 512^3 at 1 cm, frames 320x240 / 640x480, templates
4096 to 16384 particles -- every sequence's first frame step equals the
single-sequence tracker on the same inputs (sampled at 4 sequences)."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    assert torch.cuda.is_available()
    from paper_2105_05600_amd import rose
    return rose


CASES = [(256, 320, 4096, 1.0), (384, 640, 16384, 2.5), (512, 320, 10240, 4.0), (256, 640, 6144, 3.0)]


def _setup(R, i, dim, width, n, speed):
    seq = synth.room_sequence(scene_seed=1000 + i, traj_seed=2000 + i, noise_seed=3000 + i, n_frames=3, speed=speed,
                              ang_speed=0.67 * speed, width=width, height=width * 3 // 4, dim=dim)
    d0, d1 = seq.depths([0, 1])
    vol = R.Tsdf(seq.dims, seq.vox, seq.mu, seq.origin)
    p0 = seq.poses[0]
    vol.integrate(torch.from_numpy(d0).cuda(), seq.K, p0.q, p0.t)
    pst = R.pst_sample(n, 77 + i)
    return seq, vol, pst, torch.from_numpy(d1).cuda()


def test_batch_uneven_sizes_equal_single(R):
    setups = [_setup(R, i, *c) for i, c in enumerate(CASES)]
    params = [R.track_params(max_iters=20, stride=4) for _ in setups]
    # single-sequence reference (its own copy of each volume)
    refs = []
    for i, (seq, vol, pst, d1) in enumerate(setups):
        ref_vol = R.Tsdf(seq.dims, seq.vox, seq.mu, seq.origin)
        p0 = seq.poses[0]
        ref_vol.integrate(torch.from_numpy(seq.depth(0)).cuda(), seq.K, p0.q, p0.t)
        st = R.track_state(p0.q, p0.t, [0.55] * 6)
        refs.append(R.track_frame(ref_vol, d1, seq.K, pst, params[i], st))
        ref_vol.close()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = R.Batch([s[1] for s in setups], [s[0].K for s in setups], [s[2] for s in setups], params, use_graph=True)
        states = (R.TrackState * len(setups))(*[R.track_state(s[0].poses[0].q, s[0].poses[0].t, [0.55] * 6)
                                                  for s in setups])
        got = b.track([s[3] for s in setups], states, stream=stream)
        b.close()
    for g, r in zip(got, refs):
        assert g["status"] == 0 and g["aps"] == r["aps"]
        assert np.array_equal(g["t"], r["t"]) and np.array_equal(g["q"], r["q"])
