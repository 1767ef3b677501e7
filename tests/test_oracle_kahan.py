"""The "No Kahan" mode of the oracle's fitness (Sec. 5 ablation of TSDF
normalisation: the sum of psi^2 taken directly): plain binary32 summation in
point order.

Pins:
* a constructed sum: one term 1 followed by 100 000 terms 2^-26 -- each
  below half an ulp of the running sum -- leaves the plain sum at exactly 1,
  while the compensated sum is 1 + 100 000 * 2^-26 to binary64 accuracy; in
  the opposite order the plain sum keeps the small terms (within the bound);
* on random volumes the plain sum stays within the recursive-summation bound
  (m - 1) 2^-24 sum v^2 of the exact sum (math.fsum of the looked-up values,
  taken through the independent voxel-index routine), while the default sum
  (exact on the 2^-39 grid) stays within m 2^-40 of it;
* the tracker runs with the flag and still converges on the small frame.
"""
import math

import numpy as np

import synth


def _grid(orc):
    psi = np.full((8, 8, 8), 2.0 ** -13, np.float32)
    psi[0, 0, 0] = 1.0
    return psi


def test_constructed_plain_sum_loses_small_terms(orc):
    psi = _grid(orc)
    m = 100_001
    pts = np.tile(np.array([[1.5, 0.5, 0.5]], np.float32), (m, 1))
    pts[0] = (0.5, 0.5, 0.5)  # the voxel holding 1
    T = np.zeros((1, 3, 4))
    T[0, :, :3] = np.eye(3)
    exact = 1.0 + (m - 1) * 2.0 ** -26
    Fp = orc.fitness(psi, 1.0, np.zeros(3), pts, T, kahan=False, normalize=False)[0]
    Fk = orc.fitness(psi, 1.0, np.zeros(3), pts, T, kahan=True, normalize=False)[0]
    assert Fp == 1.0
    assert abs(Fk - exact) <= 1e-15 * exact
    # small terms first: the plain sum keeps them, within the bound
    rev = pts[::-1].copy()
    Fr = orc.fitness(psi, 1.0, np.zeros(3), rev, T, kahan=False, normalize=False)[0]
    assert Fr != 1.0 and abs(Fr - exact) <= (m - 1) * 2.0 ** -24 * exact
    # normalised: F = S / |O|
    Fpn = orc.fitness(psi, 1.0, np.zeros(3), pts, T, kahan=False)[0]
    assert Fpn == 1.0 / m


def test_plain_sum_within_recursive_summation_bound(orc):
    rng = np.random.default_rng(31)
    dims, vox = (32, 32, 32), 0.05
    origin = np.zeros(3, np.float32)
    psi = rng.uniform(-1, 1, (32, 32, 32)).astype(np.float32)
    pts = rng.uniform(0.0, 1.7, (5000, 3)).astype(np.float32)
    T = np.zeros((6, 3, 4))
    for i in range(6):
        T[i, :, :3] = synth.axis_angle(rng.standard_normal(3) / np.sqrt(3), rng.uniform(0, 0.1))
        T[i, :, 3] = rng.uniform(-0.05, 0.05, 3)
    idx = orc.voxel_indices(dims, vox, origin, pts, T)
    flat = psi.reshape(-1).astype(np.float64)
    Fp = orc.fitness(psi, vox, origin, pts, T, kahan=False, normalize=False)
    Fk = orc.fitness(psi, vox, origin, pts, T, kahan=True, normalize=False)
    for i in range(6):
        v = np.where(idx[i] >= 0, flat[np.maximum(idx[i], 0)], 1.0)
        exact = math.fsum(v * v)
        assert abs(Fk[i] - exact) <= len(v) * 2.0 ** -40  # the binary32 mode's exact 2^-39 grid sum
        assert abs(Fp[i] - exact) <= (len(v) - 1) * 2.0 ** -24 * exact
        assert Fp[i] != Fk[i]  # the modes really differ


def test_tracker_runs_without_kahan(orc):
    w = synth.small_frame()
    psi = synth.analytic_tsdf(w.scene, w.dims, w.vox, w.origin, w.mu)
    pst, _ = orc.pst_sample(2048, w.pst_seed)
    prev = w.fuse_poses[-1]
    res = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, np.full(6, 0.1), max_iters=10,
                          stride=w.stride, flags=orc.NO_KAHAN)
    assert res["status"] == 0
    T = orc.pose_mat(res["q"], res["t"])
    assert np.linalg.norm(T[:3, 3] - w.gt_pose.t) < 0.02
