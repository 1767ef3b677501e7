"""Pins of the oracle's geometric steps: unprojection (Eq. unproj), overlap
set (Eq. validness), fitness (Eqs. ourlh / normallh) and fusion."""
import math

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def room():
    return synth.unit_box_room(2105)


def _look(f, t):
    return synth.Pose(synth.look_rotation(f), np.asarray(t, dtype=np.float64))


# ----------------------------------------------------------- unprojection
@pytest.mark.parametrize("prec", [0, 1])
def test_unproject_lands_on_surface(orc, room, prec):
    K = synth.Intrinsics.centred(160, 120, 140.0)
    pose = _look([0.6, 0.5, 0.4], [0.01, -0.02, 0.0])
    depth = synth.render_depth(room, K, pose)
    pts = orc.unproject(depth, K, 3, prec)
    assert len(pts) == ((depth[::3, ::3] > 0).sum())
    X = pts.astype(np.float64) @ pose.R.T + pose.t
    assert np.abs(room.sdf(X)).max() < 2e-6  # binary32 storage of metre-scale points


def test_unproject_skips_invalid_and_keeps_row_major_order(orc):
    K = synth.Intrinsics.centred(8, 6, 10.0)
    d = np.arange(48, dtype=np.float32).reshape(6, 8) * 0.1
    d[2, 4] = np.nan
    d[0, 2] = -1.0
    pts = orc.unproject(d, K, 2, 0)
    expect = []
    for v in range(0, 6, 2):
        for u in range(0, 8, 2):
            z = d[v, u]
            if z > 0:
                expect.append(((u - K.cx) * z / K.fx, (v - K.cy) * z / K.fy, z))
    assert np.allclose(pts, np.array(expect, dtype=np.float32), rtol=1e-6, atol=1e-7)


# ---------------------------------------------------------------- overlap
def test_overlap_identity_keeps_interior(orc, room):
    K = synth.Intrinsics.centred(160, 120, 140.0)
    pose = _look([0.6, 0.5, 0.4], [0.0, 0.0, 0.0])
    depth = synth.render_depth(room, K, pose)
    for prec in (0, 1):
        pts = orc.unproject(depth, K, 1, prec)
        mask = orc.overlap(pts, pose.mat(), pose.mat(), K, prec)
        px = pts[:, 0] / pts[:, 2] * K.fx + K.cx
        py = pts[:, 1] / pts[:, 2] * K.fy + K.cy
        interior = (px > 0.5) & (px < K.width - 1.5) & (py > 0.5) & (py < K.height - 1.5)
        assert mask[interior].all()


def test_overlap_backward_motion_closed_form(orc, room):
    """Camera t moved back along its optical axis by delta relative to
    frame t-1: a point x maps to x' = x - (0,0,delta)... kept iff its
    projection in frame t-1 is inside the image."""
    K = synth.Intrinsics.centred(160, 120, 140.0)
    prev = _look([0.6, 0.5, 0.4], [0.05, 0.02, 0.0])
    delta = 0.08
    cur = synth.Pose(prev.R, prev.t - delta * prev.R[:, 2])  # moved backwards
    depth = synth.render_depth(room, K, cur)
    pts = orc.unproject(depth, K, 2, 0).astype(np.float64)
    mask = orc.overlap(pts, cur.mat(), prev.mat(), K, 0)
    zp = pts[:, 2] - delta
    px = K.fx * pts[:, 0] / zp + K.cx
    py = K.fy * pts[:, 1] / zp + K.cy
    expect = (zp > 0) & (px >= 0) & (px <= K.width - 1) & (py >= 0) & (py <= K.height - 1)
    margin = np.minimum.reduce([np.abs(px), np.abs(px - (K.width - 1)), np.abs(py), np.abs(py - (K.height - 1))])
    clear = margin > 1e-6
    assert 0 < expect.sum() < len(pts)  # the band is non-trivial
    assert np.array_equal(mask[clear], expect[clear])
    # moving forward instead keeps everything in view of frame t-1
    fwd = synth.Pose(prev.R, prev.t + delta * prev.R[:, 2])
    depth_f = synth.render_depth(room, K, fwd)
    pts_f = orc.unproject(depth_f, K, 2, 0)
    m_f = orc.overlap(pts_f, fwd.mat(), prev.mat(), K, 0)
    assert m_f.all()


@pytest.mark.parametrize("prec", [0, 1])
def test_overlap_prev_depth_identity_drops_exactly_the_holes(orc, room, prec):
    """Identity motion: every point projects back onto the pixel it came
    from, so the stricter test (a valid depth at the nearest pixel of frame
    t-1) keeps exactly the bounds-only set minus the points whose own pixel
    is a hole (zero, negative or NaN) of the previous depth image."""
    K = synth.Intrinsics.centred(160, 120, 140.0)
    pose = _look([0.6, 0.5, 0.4], [0.0, 0.0, 0.0])
    depth = synth.render_depth(room, K, pose)
    prev = depth.copy()
    rng = np.random.default_rng(7)
    prev[rng.random(prev.shape) < 0.3] = 0.0
    prev[40:60, 70:100] = np.nan
    prev[80:90, 10:30] = -1.0
    pts = orc.unproject(depth, K, 1, prec)
    v, u = np.nonzero(depth > 0)  # the unprojection's row-major order
    base = orc.overlap(pts, pose.mat(), pose.mat(), K, prec)
    mask = orc.overlap(pts, pose.mat(), pose.mat(), K, prec, prev_depth=prev)
    valid = prev[v, u] > 0
    assert 0 < valid.sum() < len(valid)
    assert np.array_equal(mask, base & valid)
    interior = (u > 0) & (u < K.width - 1) & (v > 0) & (v < K.height - 1)
    assert base[interior].all()
    # an all-valid previous image changes nothing
    assert np.array_equal(orc.overlap(pts, pose.mat(), pose.mat(), K, prec, prev_depth=np.ones_like(prev)), base)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shift", [3.4, 3.6])
def test_overlap_prev_depth_nearest_pixel_of_a_lateral_shift(orc, prec, shift):
    """A fronto-parallel plane at depth Z seen from frame t, whose camera
    sits (s_x, s_y) = (shift Z / fx, 0.3 Z / fy) beside frame t-1's (same
    rotation): pixel (u, v) lands at (u + shift, v + 0.3) of frame t-1, whose
    nearest pixel is (u + round(shift), v).  With an invalid column band
    [40, 50) in the previous depth image the stricter test drops exactly the
    columns u with u + round(shift) in the band; the bounds test drops
    u + shift > W - 1 and the last row (v + 0.3 > H - 1)."""
    K = synth.Intrinsics.centred(96, 64, 80.0)
    Z = 2.0
    uu, vv = np.meshgrid(np.arange(K.width), np.arange(K.height))
    u, v = uu.ravel(), vv.ravel()
    pts = np.column_stack([(u - K.cx) * Z / K.fx, (v - K.cy) * Z / K.fy, np.full(u.size, Z)]).astype(np.float32)
    prev_pose = _look([0.3, -0.8, 0.2], [0.1, 0.2, -0.05])
    cur = synth.Pose(prev_pose.R, prev_pose.t + (shift * Z / K.fx) * prev_pose.R[:, 0]
                     + (0.3 * Z / K.fy) * prev_pose.R[:, 1])
    prev = np.ones((K.height, K.width), np.float32)
    prev[:, 40:50] = 0.0
    mask = orc.overlap(pts, cur.mat(), prev_pose.mat(), K, prec, prev_depth=prev)
    base = orc.overlap(pts, cur.mat(), prev_pose.mat(), K, prec)
    in_view = (u + shift <= K.width - 1) & (v < K.height - 1)
    assert np.array_equal(base, in_view)
    near = u + int(round(shift))
    assert np.array_equal(mask, in_view & ~((near >= 40) & (near < 50)))


def test_track_frame_prev_depth_special_cases(orc):
    """Tracking with the stricter overlap test: an all-valid previous depth
    image gives the bounds-only result exactly; an all-invalid one empties
    every O_k, so every particle scores F = 1 (Eq. normallh over an empty
    set), the APS stays empty and the pose does not move."""
    w = synth.small_frame()
    nx, ny, nz = w.dims
    psi = np.ones((nz, ny, nx), np.float32)
    wt = np.zeros_like(psi)
    for p, d in zip(w.fuse_poses, w.fuse_depths):
        orc.integrate(psi, wt, w.vox, w.origin, w.mu, d, w.K, p.q, p.t, prec=orc.F32)
    pst, _ = orc.pst_sample(256, 5)
    prev = w.fuse_poses[-1]
    args = (psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, np.full(6, 0.1))
    kw = dict(max_iters=6, stride=4, prec=orc.F32)
    a = orc.track_frame(*args, **kw)
    b = orc.track_frame(*args, prev_depth=np.ones_like(w.depth), **kw)
    for key in ("q", "t", "r1", "aps", "n_overlap", "rho_iter"):
        assert np.array_equal(a[key], b[key]), key
    c = orc.track_frame(*args, prev_depth=np.zeros_like(w.depth), **kw)
    assert c["status"] == 0 and (c["n_overlap"] == 0).all() and (c["aps"] == 0).all()
    assert np.array_equal(c["t"], prev.t) and np.array_equal(c["q"], prev.q)


# ---------------------------------------------------------------- fitness
def test_fitness_plane_field_trilinear(orc):
    """psi(X) = (c - X_z)/mu is linear, so trilinear lookup is exact and a
    point set on the plane shifted by d scores F = (d/mu)^2 (Eq. normallh)."""
    nx = ny = nz = 32
    vox, mu = 0.02, 0.3
    origin = np.array([-0.32, -0.32, -0.32])
    c = 0.013
    zc = origin[2] + (np.arange(nz) + 0.5) * vox
    psi = np.broadcast_to(((c - zc) / mu)[:, None, None], (nz, ny, nx)).astype(np.float32).copy()
    rng = np.random.default_rng(0)
    xy = rng.uniform(-0.2, 0.2, size=(500, 2))
    pts = np.column_stack([xy, np.full(500, c)]).astype(np.float32)  # world = camera (identity pose)
    for d in (0.0, 0.01, -0.025, 0.07):
        T = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, d]], dtype=np.float64)
        for prec in (0, 1):
            F = orc.fitness(psi, vox, origin, pts, T[None], lookup=1, prec=prec)[0]
            assert abs(F - (d / mu) ** 2) <= 2e-6 * max((d / mu) ** 2, 1e-3)


def test_fitness_lipschitz_bound_at_true_pose(orc, room):
    """Analytic TSDF, exact surface points, nearest voxel: |psi| <= the
    centre offset sqrt(3)/2 vox / mu (the SDF is 1-Lipschitz), so
    F <= 3/4 (vox/mu)^2."""
    dims, vox, mu = (64, 64, 64), 0.02, 0.06
    origin = np.full(3, -0.64)
    psi = synth.analytic_tsdf(room, dims, vox, origin, mu)
    K = synth.Intrinsics.centred(160, 120, 140.0)
    pose = _look([0.5, 0.6, -0.3], [0.02, 0.0, 0.01])
    depth = synth.render_depth(room, K, pose)
    pts = orc.unproject(depth, K, 3, 0)
    F = orc.fitness(psi, vox, origin, pts, pose.as_3x4()[None], lookup=0, prec=1)[0]
    assert F <= 0.75 * (vox / mu) ** 2 + 1e-4
    Ft = orc.fitness(psi, vox, origin, pts, pose.as_3x4()[None], lookup=1, prec=1)[0]
    assert Ft < 2e-3
    # a 2-voxel shift along the view axis is clearly worse
    T2 = pose.as_3x4().copy()
    T2[:, 3] += 0.04 * pose.R[:, 2]
    F2 = orc.fitness(psi, vox, origin, pts, T2[None], lookup=0, prec=1)[0]
    assert F2 > 4 * F


def test_fitness_outside_grid_is_one(orc):
    psi = np.zeros((8, 8, 8), np.float32)
    pts = np.random.default_rng(1).uniform(-1, 1, (100, 3)).astype(np.float32)
    T = np.array([[1, 0, 0, 50.0], [0, 1, 0, 0], [0, 0, 1, 0]])
    for lk in (0, 1):
        for prec in (0, 1):
            assert orc.fitness(psi, 0.1, np.zeros(3), pts, T[None], lookup=lk, prec=prec)[0] == 1.0
    # no points at all: F = 1
    assert orc.fitness(psi, 0.1, np.zeros(3), np.zeros((0, 3), np.float32), T[None])[0] == 1.0


def _sum_case(seed=2, n_pts=3000, n_T=6):
    rng = np.random.default_rng(seed)
    nx, ny, nz = 24, 20, 16
    psi = rng.uniform(-1, 1, (nz, ny, nx)).astype(np.float32)
    psi[rng.random(psi.shape) < 0.1] *= 1e-6  # tiny terms, below the grid's resolution after squaring
    vox = 0.05
    origin = np.array([-0.6, -0.5, -0.4], np.float32)
    pts = rng.uniform(-0.7, 0.7, (n_pts, 3)).astype(np.float32)
    T = np.stack([np.hstack([synth.axis_angle(rng.standard_normal(3), 0.3), rng.uniform(-0.1, 0.1, (3, 1))])
                  for _ in range(n_T)])
    return psi, vox, origin, pts, T


def test_fitness_grid_sum_is_exact(orc):
    """Binary32 mode: F times |O| is the exact rational sum of the squared
    looked-up values (at the voxels the index routine reports) each rounded
    to the nearest multiple of 2^-39, ties to even, then rounded once to
    binary64 -- computed here with Fractions -- and it lies within
    |O| 2^-40 of the exactly rounded sum (math.fsum) of the squares."""
    from fractions import Fraction
    psi, vox, origin, pts, T = _sum_case()
    nz, ny, nx = psi.shape
    F = orc.fitness(psi, vox, origin, pts, T, lookup=0, prec=1)
    idx = orc.voxel_indices((nx, ny, nz), vox, origin, pts, T)
    flat = psi.ravel().astype(np.float64)
    m = len(pts)
    for i in range(len(T)):
        v = np.where(idx[i] >= 0, flat[np.maximum(idx[i], 0)], 1.0)
        q = sum(round(Fraction(float(x)) ** 2 * 2 ** 39) for x in v)  # round(): nearest, ties to even
        assert F[i] == (float(q) * 2.0 ** -39) / m
        assert abs(F[i] * m - math.fsum(v * v)) <= m * 2.0 ** -40


def test_fitness_grid_sum_ignores_point_order(orc):
    """Binary32 mode: any permutation of the points gives the same F bit
    for bit (the grid sum is exact); binary64 mode's compensated sum need
    not, but stays within a few ulps."""
    psi, vox, origin, pts, T = _sum_case(seed=5, n_pts=2000, n_T=4)
    perm = np.random.default_rng(9).permutation(len(pts))
    for lk in (0, 1):
        a = orc.fitness(psi, vox, origin, pts, T, lookup=lk, prec=1)
        b = orc.fitness(psi, vox, origin, pts[perm], T, lookup=lk, prec=1)
        assert np.array_equal(a, b)
        a64 = orc.fitness(psi, vox, origin, pts, T, lookup=lk, prec=0)
        b64 = orc.fitness(psi, vox, origin, pts[perm], T, lookup=lk, prec=0)
        assert np.allclose(a64, b64, rtol=1e-14, atol=0)


def test_fitness_binary64_sum_is_compensated(orc):
    """Binary64 mode: with the identity pose and points at voxel centres
    (the voxel is unambiguous in either precision), F times |O| equals the
    exactly rounded sum (math.fsum) of the squares within 1e-15 relative
    (Neumaier compensation)."""
    rng = np.random.default_rng(3)
    nx, ny, nz = 24, 20, 16
    psi = rng.uniform(-1, 1, (nz, ny, nx)).astype(np.float32)
    vox = 0.0625
    origin = np.zeros(3, np.float32)
    ijk = np.stack([rng.integers(0, n, 5000) for n in (nx, ny, nz)], axis=1)
    pts = ((ijk + 0.5) * vox).astype(np.float32)
    T = np.hstack([np.eye(3), np.zeros((3, 1))])[None]
    F = orc.fitness(psi, vox, origin, pts, T, lookup=0, prec=0)[0]
    v = psi[ijk[:, 2], ijk[:, 1], ijk[:, 0]].astype(np.float64)
    exact = math.fsum(v * v) / len(pts)
    assert abs(F - exact) <= 1e-15 * exact


def test_exp_rho_matches_exp(orc):
    """The oracle's exp (Cody-Waite reduction, Taylor polynomial, 2^k
    scaling) is within one ulp of math.exp over the likelihood range
    (rho = exp(-F / tau), F >= 0) and exact at 0."""
    rng = np.random.default_rng(4)
    xs = np.concatenate([-rng.uniform(0, 1, 4000), -rng.uniform(0, 50, 2000), -rng.uniform(0, 745, 500),
                         -np.arange(0, 40) * math.log(2), [-1e-300, -0.5, -1.0]])
    got = orc.exp_rho(xs)
    for x, g in zip(xs, got):
        e = math.exp(x)
        assert abs(g - e) <= math.ulp(e), (x, g, e)
    assert orc.exp_rho([0.0])[0] == 1.0 and orc.exp_rho([-2000.0])[0] == 0.0


def test_voxel_indices_are_floor_of_voxel_coordinate(orc):
    """Indices (binary32 decision) agree with the binary64 definition
    floor((R x + t - origin) / vox) wherever the coordinate is not within
    1e-4 voxel of a cell boundary."""
    rng = np.random.default_rng(3)
    dims = (40, 30, 20)
    vox = 0.025
    origin = np.array([-0.5, -0.4, -0.25], np.float32)
    pts = rng.uniform(-0.6, 0.6, (2000, 3)).astype(np.float32)
    T = np.hstack([synth.axis_angle([1, 2, 3], 0.4), [[0.01], [-0.02], [0.03]]])
    idx = orc.voxel_indices(dims, vox, origin, pts, T[None])[0]
    g = ((pts.astype(np.float64) @ T[:, :3].T + T[:, 3]) - origin.astype(np.float64)) / vox
    fl = np.floor(g).astype(np.int64)
    inside = np.all((fl >= 0) & (fl < np.array(dims)), axis=1)
    expect = np.where(inside, (fl[:, 2] * dims[1] + fl[:, 1]) * dims[0] + fl[:, 0], -1)
    clear = np.all(np.abs(g - np.round(g)) > 1e-4, axis=1)
    assert clear.mean() > 0.99
    assert np.array_equal(idx[clear], expect[clear])


# ---------------------------------------------------------------- fusion
@pytest.mark.parametrize("prec", [0, 1])
def test_integrate_fronto_parallel_plane(orc, prec):
    """A camera at the origin looking along +z at the wall z = D: along a
    voxel column near the optical axis, every voxel that projects into the
    image with D - z >= -mu holds min(1, (D - z)/mu) after one frame,
    W = 1; voxels out of view or further behind are untouched."""
    scene = synth.Scene(np.array([-3.0, -3.0, -3.0]), np.array([3.0, 3.0, 0.553]))
    K = synth.Intrinsics.centred(64, 48, 60.0)
    pose = synth.Pose(np.eye(3), np.zeros(3))
    depth = synth.render_depth(scene, K, pose)
    assert np.allclose(depth, 0.553, atol=1e-6)
    n, vox, mu = 32, 0.02, 0.06
    origin = np.array([-0.32, -0.32, 0.0], np.float32)
    psi = np.ones((n, n, n), np.float32)
    w = np.zeros_like(psi)
    orc.integrate(psi, w, vox, origin, mu, depth, K, [1, 0, 0, 0], [0, 0, 0], prec=prec)
    i = j = 16  # voxel column whose centre is at x = y = 0.01
    for k in range(n):
        z = origin[2] + (k + 0.5) * vox
        xc = origin[0] + (i + 0.5) * vox
        u = math.floor(K.fx * xc / z + K.cx + 0.5)
        sdf = 0.553 - z
        if 0 <= u < K.width and sdf >= -mu:
            assert w[k, j, i] == 1.0
            assert abs(psi[k, j, i] - min(1.0, sdf / mu)) < 1e-5
        else:
            assert w[k, j, i] == 0.0 and psi[k, j, i] == 1.0


def test_integrate_weight_cap_and_fixed_point(orc):
    scene = synth.Scene(np.array([-3.0, -3.0, -3.0]), np.array([3.0, 3.0, 0.4]))
    K = synth.Intrinsics.centred(32, 24, 30.0)
    depth = synth.render_depth(scene, K, synth.Pose(np.eye(3), np.zeros(3)))
    n = 16
    psi = np.ones((n, n, n), np.float32)
    w = np.zeros_like(psi)
    once = None
    for rep in range(6):
        orc.integrate(psi, w, 0.04, np.array([-0.32, -0.32, 0.0]), 0.1, depth, K, [1, 0, 0, 0], [0, 0, 0],
                      w_max=4.0, prec=1)
        if rep == 0:
            once = psi.copy()
    seen = w > 0
    assert seen.any() and np.all(w[seen] == 4.0)
    assert np.allclose(psi[seen], once[seen], atol=2e-7)  # the same frame is a fixed point


def test_integrate_zero_crossing_near_surface(orc, room):
    """Single noise-free frame: trilinear reads of the fused TSDF at the
    frame's own surface points are near zero (projective-distance and
    nearest-pixel error only)."""
    dims, vox, mu = (64, 64, 64), 0.02, 0.06
    origin = np.full(3, -0.64)
    K = synth.Intrinsics.centred(160, 120, 140.0)
    pose = _look([0.6, 0.5, 0.4], [0.0, 0.01, 0.0])
    depth = synth.render_depth(room, K, pose)
    psi = np.ones((64, 64, 64), np.float32)
    w = np.zeros_like(psi)
    orc.integrate(psi, w, vox, origin, mu, depth, K, pose.q, pose.t, prec=0)
    pts = orc.unproject(depth, K, 3, 0)
    F = orc.fitness(psi, vox, origin, pts, pose.as_3x4()[None], lookup=1, prec=0)[0]
    assert F < 0.02
