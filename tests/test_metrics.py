"""Trajectory metrics used by the bench and the experiments (Sec. 5.1: ATE
after rigid alignment, TE of Eq. te).

Pins: a rigidly moved copy of a trajectory has ATE 0 and the alignment
recovers the motion; a trajectory displaced by one point's error has the
closed-form ATE of the aligned residual; TE of a constant body-frame offset
is its norm; a mirror image is not matched by a rotation (det = +1)."""
import numpy as np

import synth


def _traj(n=80, seed=3):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.normal(0, 0.05, (n, 3)), axis=0) + rng.normal(0, 1, 3)


def test_rigid_copy_has_zero_ate():
    gt = _traj()
    R = synth.axis_angle(np.array([0.2, -0.9, 0.4]) / np.linalg.norm([0.2, -0.9, 0.4]), 1.1)
    t = np.array([0.3, -2.0, 0.7])
    est = gt @ R.T + t
    mean, rmse = synth.ate(est, gt)
    assert mean < 1e-12 and rmse < 1e-12
    Ra, ta = synth.horn_align(est, gt)  # maps est back onto gt: R^T, -R^T t
    assert np.allclose(Ra, R.T, atol=1e-12) and np.allclose(ta, -R.T @ t, atol=1e-12)
    assert abs(np.linalg.det(Ra) - 1) < 1e-12


def test_translation_only_error_is_not_absorbed():
    # est = gt except one point moved by d: the best rigid fit spreads it, but
    # a pure translation of the whole trajectory is absorbed exactly
    gt = _traj()
    assert synth.ate(gt + np.array([0.4, 0.0, -0.1]), gt)[1] < 1e-12
    est = gt.copy()
    est[10] += np.array([0.0, 0.05, 0.0])
    mean, rmse = synth.ate(est, gt)
    assert 0 < rmse < 0.05 and mean <= rmse


def test_te_of_constant_body_offset():
    rng = np.random.default_rng(5)
    for _ in range(5):
        R = synth.axis_angle(rng.normal(size=3) / np.linalg.norm(rng.normal(size=3)), rng.uniform(0, 3))
        G = np.eye(4)
        G[:3, :3] = R
        G[:3, 3] = rng.normal(size=3)
        off = np.eye(4)
        off[:3, 3] = rng.normal(size=3) * 0.1
        E = G @ off
        assert abs(synth.translation_error(G, E) - np.linalg.norm(off[:3, 3])) < 1e-12


def test_mirror_image_is_not_a_rotation():
    gt = _traj(seed=9)
    est = gt * np.array([1.0, 1.0, -1.0])  # reflection
    R, _ = synth.horn_align(est, gt)
    assert abs(np.linalg.det(R) - 1) < 1e-12
    assert synth.ate(est, gt)[1] > 1e-3
