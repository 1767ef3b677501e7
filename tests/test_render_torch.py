"""The batched torch depth renderer (used for training data on the GPU)
reproduces the numpy renderer: noise-free frames agree to rounding on a
procedural room (boxes, cylinders, spheres) and on the small frame's
sphere room; the noise follows N(0, (k z^2)^2) and the validity range."""
import numpy as np
import torch

import synth
from synth.gpu_render import render_depths


def test_noise_free_frames_match_numpy():
    seq = synth.configs.ablation_sequence("6d", 64010, 6, 160, 120)
    poses = seq.poses[:6]
    ref = np.stack([synth.render_depth(seq.scene, seq.K, p, seq.zmin, seq.zmax) for p in poses])
    got = render_depths(seq.scene, seq.K, poses, seq.zmin, seq.zmax, device="cpu").numpy()
    assert np.array_equal(got > 0, ref > 0)
    assert np.max(np.abs(got - ref)) <= 1e-6
    assert np.mean(got == ref) > 0.999
    w = synth.small_frame()
    ref = synth.render_depth(w.scene, w.K, w.gt_pose)
    got = render_depths(w.scene, w.K, [w.gt_pose], device="cpu")[0].numpy()
    assert np.max(np.abs(got - ref)) <= 1e-6


def test_noise_model():
    seq = synth.configs.ablation_sequence("6d", 64020, 2, 160, 120)
    clean = render_depths(seq.scene, seq.K, seq.poses[:2], device="cpu").double()
    noisy = render_depths(seq.scene, seq.K, seq.poses[:2], noise_seed=7, noise_k=0.002, device="cpu").double()
    again = render_depths(seq.scene, seq.K, seq.poses[:2], noise_seed=7, noise_k=0.002, device="cpu").double()
    assert torch.equal(noisy, again)  # seeded
    m = (clean > 0.3) & (clean < 5.5) & (noisy > 0)
    r = ((noisy - clean) / (0.002 * clean * clean))[m]
    assert abs(float(r.mean())) < 0.02 and abs(float(r.std()) - 1.0) < 0.02
    cut = render_depths(seq.scene, seq.K, seq.poses[:2], zmin=1.0, zmax=3.0, device="cpu")
    v = cut[cut > 0]
    assert float(v.min()) > 1.0 and float(v.max()) < 3.0
