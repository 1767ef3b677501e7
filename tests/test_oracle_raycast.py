"""Pins of the oracle's TSDF raycast (the model rendered at a pose)."""
import numpy as np

import synth


def test_raycast_matches_analytic_render(orc):
    """Analytic TSDF of the box room: the rendered depth is within half a
    voxel of the closed-form ray intersection (trilinear + linear
    interpolation of the crossing)."""
    room = synth.unit_box_room(2105)
    dims, vox, mu = (64, 64, 64), 0.02, 0.06
    origin = np.full(3, -0.64)
    psi = synth.analytic_tsdf(room, dims, vox, origin, mu)
    K = synth.Intrinsics.centred(40, 30, 35.0)
    pose = synth.Pose(synth.look_rotation([0.6, 0.5, 0.4]), np.array([0.01, -0.02, 0.0]))
    d = orc.raycast(psi, vox, origin, pose.q, pose.t, K, near=0.05, far=2.0, step=0.01)
    ref = synth.render_depth(room, K, pose)
    m = (d > 0) & (ref > 0)
    assert m.mean() > 0.99
    assert np.abs(d - ref)[m].max() <= vox / 2


def test_raycast_plane_is_exact_and_misses_are_zero(orc):
    """A plane field psi = (c - z)/mu is linear inside the band, so the
    interpolated crossing is the plane itself; rays that leave the grid
    without a crossing return 0."""
    n, vox, mu = 32, 0.02, 0.1
    origin = np.array([-0.32, -0.32, 0.0])
    c = 0.437
    zc = origin[2] + (np.arange(n) + 0.5) * vox
    psi = np.broadcast_to(np.clip((c - zc) / mu, -1, 1)[:, None, None], (n, n, n)).astype(np.float32).copy()
    K = synth.Intrinsics.centred(16, 12, 20.0)
    d = orc.raycast(psi, vox, origin, [1, 0, 0, 0], [0, 0, 0], K, near=0.05, far=1.0, step=0.013)
    assert np.all(np.abs(d - c) < 1e-6)
    d_far = orc.raycast(psi, vox, origin, [1, 0, 0, 0], [0, 0, 0], K, near=0.05, far=0.3, step=0.013)
    assert np.all(d_far == 0)


def test_proposal_features_closed_forms(orc):
    """Constant frames: the residual is the clamped depth difference on every
    low-res pixel, 0 where either depth is missing; the velocity follows the
    residual block and the rest is zero padding."""
    depth = np.full((240, 320), 2.0, np.float32)
    render = np.full((30, 40), 1.75, np.float32)
    render[3, 7] = 0.0          # no model surface there
    depth[8 * 5 + 4, 8 * 9 + 4] = 0.0  # no measurement at low-res pixel (9, 5)
    depth[8 * 1 + 4, 8 * 2 + 4] = 3.0  # residual 1.25 m -> clamped to 0.5
    vel = [0.1, -0.2, 0.3, 1.0, 2.0, -3.0]
    f = orc.proposal_features(depth, render, 8, vel, 1216)
    res = f[:1200].reshape(30, 40)
    expect = np.full((30, 40), np.float32(2.0) - np.float32(1.75))
    expect[3, 7] = 0.0
    expect[5, 9] = 0.0
    expect[1, 2] = 0.5
    assert np.array_equal(res, expect)
    assert np.array_equal(f[1200:1206], np.array(vel, np.float32))
    assert np.all(f[1206:] == 0)
