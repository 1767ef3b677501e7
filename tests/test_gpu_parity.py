"""GPU path (librose through its C ABI) against the CPU oracle, element by
element on the same seeded inputs.

Bars: bit-exact for the PST template, binary64 particle poses, unprojected
points, overlap masks and voxel indices (integer or exactly specified
results); bit-exact for NEAREST fitness (same voxels, sums exact on the
2^-39 grid on both sides, one rounding to binary32), relative 1e-5 for
TRILINEAR fitness (the oracle interpolates in binary64); 1e-4 m / 1e-4 rad
on tracked poses.
"""
import math

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2105_05600_amd import rose
    return rose


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def oracle_volume(orc, w):
    """The oracle's binary32 fusion of a small frame's fusion depths."""
    nx, ny, nz = w.dims
    psi = np.ones((nz, ny, nx), np.float32)
    wt = np.zeros_like(psi)
    for p, d in zip(w.fuse_poses, w.fuse_depths):
        orc.integrate(psi, wt, w.vox, w.origin, w.mu, d, w.K, p.q, p.t, prec=orc.F32)
    return psi


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30))


def _rot_err(qa, qb):
    Ra, Rb = synth.quat_to_mat(qa), synth.quat_to_mat(qb)
    c = np.clip((np.trace(Ra.T @ Rb) - 1) / 2, -1, 1)
    return math.acos(c)


# ------------------------------------------------------------------- a1 PST
@pytest.mark.parametrize("n,seed", [(1, 1), (5, 3), (1023, 5600), (10240, 5600), (16384, 77), (65536, 9)])
def test_pst_sample_bit_exact(R, orc, n, seed):
    g = host(R.pst_sample(n, seed))
    o, _ = orc.pst_sample(n, seed)
    assert g.dtype == np.float32 and g.shape == (n, 6)
    assert np.array_equal(g.view(np.uint32), o.view(np.uint32))


# --------------------------------------------------------- a4 particle poses
def test_particle_poses_bit_exact(R, orc):
    rng = np.random.default_rng(11)
    pst, _ = orc.pst_sample(1000, 9)
    for _ in range(3):
        q = synth.mat_to_quat(synth.axis_angle(rng.standard_normal(3), rng.uniform(0, 3)))
        t = rng.uniform(-3, 3, 3)
        r = rng.uniform(0.001, 1.0, 6)
        g = host(R.particle_poses(q, t, r, dev(pst)))
        o = orc.particle_poses(q, t, r, pst)
        assert np.array_equal(g.view(np.uint64), o.view(np.uint64))


# ------------------------------------------------------ a2 unprojection
@pytest.mark.parametrize("W,H,f,stride", [(160, 120, 140.0, 3), (640, 480, 525.0, 4), (97, 61, 80.0, 7),
                                          (64, 48, 60.0, 1)])
def test_unproject_bit_exact(R, orc, W, H, f, stride):
    room = synth.unit_box_room(2105)
    K = synth.Intrinsics.centred(W, H, f)
    pose = synth.Pose(synth.look_rotation([0.6, 0.5, 0.4]), np.array([0.01, -0.02, 0.0]))
    depth = synth.render_depth(room, K, pose, noise_seed=4, noise_k=0.002)
    depth[::5, ::3] = 0.0  # holes
    g = host(R.depth_unproject(dev(depth), K, stride))
    o = orc.unproject(depth, K, stride, orc.F32)
    assert g.shape == o.shape
    assert np.array_equal(g.view(np.uint32), o.view(np.uint32))


def test_unproject_tiled_order_is_a_permutation(R, orc):
    """The tracker's 8x8-tile sample order lists exactly the oracle's
    points, permuted tile by tile."""
    room = synth.unit_box_room(2105)
    K = synth.Intrinsics.centred(101, 77, 90.0)
    pose = synth.Pose(synth.look_rotation([0.6, 0.5, 0.4]), np.array([0.01, -0.02, 0.0]))
    depth = synth.render_depth(room, K, pose)
    depth[::3, ::5] = 0.0
    stride = 3
    g = host(R.depth_unproject(dev(depth), K, stride, tiled=True))
    o = orc.unproject(depth, K, stride, orc.F32)
    su, sv = -(-K.width // stride), -(-K.height // stride)
    row_major = [(uu, vv) for vv in range(sv) for uu in range(su) if depth[vv * stride, uu * stride] > 0]
    index = {p: i for i, p in enumerate(row_major)}
    ntx, nty = -(-su // 8), -(-sv // 8)
    tiled = []
    for t in range(ntx * nty):
        for e in range(64):
            uu, vv = (t % ntx) * 8 + e % 8, (t // ntx) * 8 + e // 8
            if uu < su and vv < sv and depth[vv * stride, uu * stride] > 0:
                tiled.append(index[(uu, vv)])
    assert np.array_equal(g.view(np.uint32), o[tiled].view(np.uint32))


# --------------------------------------------------------- a3 overlap mask
def test_overlap_mask_bit_exact(R, orc):
    room = synth.unit_box_room(2105)
    K = synth.Intrinsics.centred(160, 120, 140.0)
    rng = np.random.default_rng(5)
    prev = synth.Pose(synth.look_rotation([0.6, 0.5, 0.4]), np.array([0.01, -0.02, 0.0]))
    for _ in range(4):
        cur = synth.Pose(synth.axis_angle(rng.standard_normal(3), 0.15) @ prev.R, prev.t + rng.uniform(-0.1, 0.1, 3))
        depth = synth.render_depth(room, K, cur)
        pts = orc.unproject(depth, K, 1, orc.F32)
        g = host(R.overlap_mask(dev(pts), (cur.q, cur.t), (prev.q, prev.t), K))
        o = orc.overlap(pts, orc.pose_mat(cur.q, cur.t), orc.pose_mat(prev.q, prev.t), K, orc.F32)
        assert 0 < o.sum() < len(o)
        assert np.array_equal(g, o)


def test_overlap_mask_prev_depth_bit_exact(R, orc):
    """The stricter overlap test (valid depth at the nearest pixel of frame
    t-1) on the GPU equals the oracle's mask bit for bit, with holes (zero,
    negative, NaN) in the previous depth image."""
    room = synth.unit_box_room(2105)
    K = synth.Intrinsics.centred(160, 120, 140.0)
    rng = np.random.default_rng(9)
    prev = synth.Pose(synth.look_rotation([0.6, 0.5, 0.4]), np.array([0.01, -0.02, 0.0]))
    prev_depth = synth.render_depth(room, K, prev)
    prev_depth[rng.random(prev_depth.shape) < 0.25] = 0.0
    prev_depth[30:50, 20:60] = np.nan
    prev_depth[90:100, 100:140] = -2.0
    for _ in range(4):
        cur = synth.Pose(synth.axis_angle(rng.standard_normal(3), 0.15) @ prev.R, prev.t + rng.uniform(-0.1, 0.1, 3))
        depth = synth.render_depth(room, K, cur)
        pts = orc.unproject(depth, K, 1, orc.F32)
        g = host(R.overlap_mask(dev(pts), (cur.q, cur.t), (prev.q, prev.t), K, prev_depth=dev(prev_depth)))
        o = orc.overlap(pts, orc.pose_mat(cur.q, cur.t), orc.pose_mat(prev.q, prev.t), K, orc.F32,
                        prev_depth=prev_depth)
        b = orc.overlap(pts, orc.pose_mat(cur.q, cur.t), orc.pose_mat(prev.q, prev.t), K, orc.F32)
        assert 0 < o.sum() < b.sum()
        assert np.array_equal(g, o)


# ------------------------------------------------- a5 voxel indices, fitness
def stored_values(psi, fmt):
    """psi (binary32) as the storage format holds it, from the formats'
    definitions: binary16 round-to-nearest-even; SNORM16 code
    round(clamp(psi) * 32767) read back as code * (1/32767) in binary32."""
    psi = np.asarray(psi, np.float32)
    if fmt == 0:
        return psi.copy()
    if fmt == 1:
        return psi.astype(np.float16).astype(np.float32)
    code = np.rint(np.clip(psi, -1, 1) * np.float32(32767)).astype(np.int16)
    return code.astype(np.float32) * np.float32(1.0 / 32767.0)


def _random_volume(R, rng, dims, vox, origin, fmt=0):
    """A random volume loaded on the GPU, and the oracle's copy of it made
    on the host (the export is checked against that copy, never used)."""
    nx, ny, nz = dims
    psi = rng.uniform(-1, 1, (nz, ny, nx)).astype(np.float32)
    psi[rng.random((nz, ny, nx)) < 0.2] = 1.0
    vol = R.Tsdf(dims, vox, 3 * vox, origin, fmt=fmt)
    vol.load(dev(psi.ravel()))
    ref = stored_values(psi, fmt)
    gpsi, _ = vol.export()
    assert np.array_equal(host(gpsi).view(np.uint32), ref.view(np.uint32))
    return vol, ref


def _random_poses(rng, n, spread=0.3):
    T = np.zeros((n, 3, 4), np.float32)
    for i in range(n):
        T[i, :, :3] = synth.axis_angle(rng.standard_normal(3), rng.uniform(0, spread))
        T[i, :, 3] = rng.uniform(-0.1, 0.1, 3)
    return T


def test_voxel_indices_bit_exact(R, orc):
    rng = np.random.default_rng(6)
    dims, vox, origin = (24, 16, 32), 0.05, (-0.6, -0.4, -0.8)
    vol, _ = _random_volume(R, rng, dims, vox, origin)
    pts = rng.uniform(-0.6, 0.6, (777, 3)).astype(np.float32)
    T = _random_poses(rng, 9)
    g = host(R.voxel_indices(vol, dev(pts), dev(T)))
    o = orc.voxel_indices(dims, vox, np.array(origin, np.float32), pts, T.astype(np.float64))
    assert (o >= 0).mean() > 0.3 and (o < 0).any()
    assert np.array_equal(g, o)


@pytest.mark.parametrize("shape", [(2, 4), (4, 4), (4, 8), (8, 2), (8, 4), (64, 4), (64, 8), (64, 16)])
def test_fitness_shapes_parity(R, orc, shape):
    rng = np.random.default_rng(31)
    dims, vox, origin = (32, 24, 16), 0.04, (-0.64, -0.48, -0.32)
    vol, psi = _random_volume(R, rng, dims, vox, origin)
    pts = rng.uniform(-0.7, 0.7, (2999, 3)).astype(np.float32)
    T = _random_poses(rng, 77)
    try:
        R.set_fitness_shape(*shape)
        F, _ = R.fitness_eval(vol, dev(pts), dev(T), 0)
        F = host(F)
    finally:
        R.set_fitness_shape(4, 2)
    Fo = orc.fitness(psi, vox, np.array(origin, np.float32), pts, T.astype(np.float64), lookup=0, prec=orc.F32)
    assert np.array_equal(F, Fo.astype(np.float32))


@pytest.mark.parametrize("fmt", [0, 1])
def test_fitness_all_ones_bricks(R, orc, fmt):
    """Bricks holding only +1 are skipped by the points-across kernel (the
    value is known): a volume with every other 8x8x8 brick set to +1 gives
    the oracle's fitness bit for bit in every shape, and after the psi
    buffer is overwritten directly, tsdf_rescan brings the bits up to date."""
    rng = np.random.default_rng(41)
    dims, vox, origin = (32, 24, 16), 0.04, (-0.64, -0.48, -0.32)
    nx, ny, nz = dims
    psi = rng.uniform(-1, 1, (nz, ny, nx)).astype(np.float32)
    k, j, i = np.meshgrid(np.arange(nz) // 8, np.arange(ny) // 8, np.arange(nx) // 8, indexing="ij")
    psi[(k + j + i) % 2 == 0] = 1.0
    vol = R.Tsdf(dims, vox, 3 * vox, origin, fmt=fmt)
    vol.load(dev(psi.ravel()))
    ref = stored_values(psi, fmt)
    pts = rng.uniform(-0.7, 0.7, (2999, 3)).astype(np.float32)
    T = _random_poses(rng, 67)
    Fo = orc.fitness(ref, vox, np.array(origin, np.float32), pts, T.astype(np.float64), lookup=0, prec=orc.F32)
    try:
        for shape in ((4, 4), (4, 8), (8, 4), (64, 8)):
            vol.set_fitness_shape(*shape)
            F, _ = R.fitness_eval(vol, dev(pts), dev(T), 0)
            assert np.array_equal(host(F), Fo.astype(np.float32)), shape
        # overwrite psi in place (all zeros: the same bytes in any layout), then rescan
        vol.psi.zero_()
        vol.rescan()
        Fz = orc.fitness(np.zeros_like(ref), vox, np.array(origin, np.float32), pts, T.astype(np.float64),
                         lookup=0, prec=orc.F32)
        vol.set_fitness_shape(4, 4)
        F, _ = R.fitness_eval(vol, dev(pts), dev(T), 0)
        assert np.array_equal(host(F), Fz.astype(np.float32))
    finally:
        vol.close()


@pytest.mark.parametrize("fmt", [0, 1, 2])
@pytest.mark.parametrize("lookup", [0, 1])
@pytest.mark.parametrize("n,m", [(1, 1), (5, 63), (67, 65), (130, 3001), (9, 0)])
def test_fitness_parity(R, orc, fmt, lookup, n, m):
    rng = np.random.default_rng(100 + n + m)
    dims, vox, origin = (32, 24, 16), 0.04, (-0.64, -0.48, -0.32)
    vol, psi = _random_volume(R, rng, dims, vox, origin, fmt)
    pts = rng.uniform(-0.7, 0.7, (m, 3)).astype(np.float32)
    T = _random_poses(rng, n)
    F, rho = R.fitness_eval(vol, dev(pts), dev(T), lookup)
    F, rho = host(F), host(rho)
    Fo = orc.fitness(psi, vox, np.array(origin, np.float32), pts, T.astype(np.float64), lookup=lookup, prec=orc.F32)
    assert _rel(F, Fo) <= 1e-5
    if lookup == 0:
        assert np.array_equal(F, Fo.astype(np.float32))
    assert _rel(rho, np.exp(-Fo)) <= 1e-5
    if m == 0:
        assert np.all(F == 1.0)


@pytest.mark.parametrize("fmt", [0, 1, 2])
@pytest.mark.parametrize("lookup", [0, 1])
@pytest.mark.parametrize("n,m", [(1, 1), (63, 65), (64, 64), (65, 3001), (130, 63), (9, 0)])
def test_fitness_parity_particle_per_lane(R, orc, fmt, lookup, n, m):
    """The one-particle-per-lane shape (64, 8): particle counts around the
    64-lane wave and point counts around the 64-point step and its 8-point
    sub-steps, every storage format and lookup."""
    rng = np.random.default_rng(300 + n + m)
    dims, vox, origin = (32, 24, 16), 0.04, (-0.64, -0.48, -0.32)
    vol, psi = _random_volume(R, rng, dims, vox, origin, fmt)
    pts = rng.uniform(-0.7, 0.7, (m, 3)).astype(np.float32)
    T = _random_poses(rng, n)
    try:
        R.set_fitness_shape(64, 8)
        F, rho = R.fitness_eval(vol, dev(pts), dev(T), lookup)
        F, rho = host(F), host(rho)
    finally:
        R.set_fitness_shape(4, 2)
    Fo = orc.fitness(psi, vox, np.array(origin, np.float32), pts, T.astype(np.float64), lookup=lookup, prec=orc.F32)
    assert _rel(F, Fo) <= 1e-5
    if lookup == 0:
        assert np.array_equal(F, Fo.astype(np.float32))
    assert _rel(rho, np.exp(-Fo)) <= 1e-5
    if m == 0:
        assert np.all(F == 1.0)


@pytest.fixture(scope="module")
def room_frame(R, orc):
    """Frame 0 of the 640x480 room sequence fused into a 512^3 volume at
    1 cm twice: on the GPU (vol) and by the oracle (psi, w, the oracle's
    inputs); frame 1 is tracked against it."""
    seq = synth.room_sequence(n_frames=3)
    d0, d1 = seq.depths([0, 1])
    vol = R.Tsdf(seq.dims, seq.vox, seq.mu, seq.origin)
    p0 = seq.poses[0]
    vol.integrate(dev(d0), seq.K, p0.q, p0.t)
    nx, ny, nz = seq.dims
    psi = np.ones((nz, ny, nx), np.float32)
    w = np.zeros_like(psi)
    orc.integrate(psi, w, seq.vox, seq.origin, seq.mu, d0, seq.K, p0.q, p0.t, prec=orc.F32)
    return seq, vol, psi, w, d0, d1


def test_fitness_full_size_sampled(R, orc, room_frame):
    """10240 poses x all points of a 640x480 frame (stride 4) on the
    512^3 volume, in the launch shape the tracker uses; 24 sampled
    particles are recomputed by the oracle one by one."""
    seq, vol, psi, _, _, d1 = room_frame
    rng = np.random.default_rng(8)
    pts = orc.unproject(d1, seq.K, seq.stride, orc.F32)
    assert len(pts) > 10000
    p0 = seq.poses[0]
    T = np.repeat(p0.as_3x4()[None], 10240, 0)
    T[:, :, :3] = np.einsum("nij,jk->nik", np.stack([synth.axis_angle(rng.standard_normal(3), rng.uniform(0, 0.1))
                                                     for _ in range(10240)]), p0.R)
    T[:, :, 3] += rng.uniform(-0.1, 0.1, (10240, 3))
    T = T.astype(np.float32)
    pick = np.concatenate([[0, 10239], rng.choice(10240, 22, replace=False)])
    for lookup in (0, 1):
        Fo = orc.fitness(psi, seq.vox, seq.origin.astype(np.float32), pts, T[pick].astype(np.float64), lookup=lookup,
                         prec=orc.F32)
        # every launch shape the autotuner may pick for the bench
        for shape in ((2, 4), (4, 2), (4, 4), (4, 8), (8, 2), (8, 4), (64, 4), (64, 8), (64, 16)):
            try:
                R.set_fitness_shape(*shape)
                F, _ = R.fitness_eval(vol, dev(pts), dev(T), lookup)
                F = host(F)
            finally:
                R.set_fitness_shape(4, 2)
            assert _rel(F[pick], Fo) <= 1e-5, (lookup, shape)
            if lookup == 0:
                assert np.array_equal(F[pick], Fo.astype(np.float32)), shape
            assert np.all((F >= 0) & (F <= 1))


# ------------------------------------------------------------ a8 fusion
@pytest.mark.parametrize("fmt", [0])
def test_integrate_parity_small(R, orc, fmt):
    w = synth.small_frame()
    nx, ny, nz = w.dims
    vol = R.Tsdf(w.dims, w.vox, w.mu, w.origin, fmt=fmt)
    psi = np.ones((nz, ny, nx), np.float32)
    wt = np.zeros_like(psi)
    for p, d in zip(w.fuse_poses, w.fuse_depths):
        vol.integrate(dev(d), w.K, p.q, p.t)
        orc.integrate(psi, wt, w.vox, w.origin, w.mu, d, w.K, p.q, p.t, prec=orc.F32)
    gp, gw = vol.export()
    gp, gw = host(gp), host(gw)
    assert np.array_equal(gw, wt)
    assert np.array_equal(gp.view(np.uint32), psi.view(np.uint32))


def test_integrate_parity_full_size(R, orc, room_frame):
    """Frame 0 of the 640x480 room sequence fused into the 512^3 volume:
    weights equal and psi bit-identical to the oracle's binary32 fusion."""
    seq, vol, full_psi, full_w, d0, _ = room_frame
    gp, gw = vol.export()
    gp, gw = host(gp), host(gw)
    assert (full_w > 0).sum() > 1_000_000
    assert np.array_equal(gw, full_w)
    assert np.array_equal(gp.view(np.uint32), full_psi.view(np.uint32))


# --------------------------------------------------------- whole frame
@pytest.fixture(scope="module")
def small_gpu(R, orc):
    """The small frame's volume fused on the GPU (vol) and by the oracle
    (psi, the oracle's input)."""
    w = synth.small_frame()
    vol = R.Tsdf(w.dims, w.vox, w.mu, w.origin)
    for p, d in zip(w.fuse_poses, w.fuse_depths):
        vol.integrate(dev(d), w.K, p.q, p.t)
    psi = oracle_volume(orc, w)
    pst, _ = orc.pst_sample(w.n_particles, w.pst_seed)
    return w, vol, psi, pst


@pytest.mark.parametrize("lookup", [0, 1])
@pytest.mark.parametrize("r0", [0.1, 0.55])
def test_track_frame_parity(R, orc, small_gpu, lookup, r0):
    w, vol, psi, pst = small_gpu
    prev = w.fuse_poses[-1]
    params = R.track_params(max_iters=w.iters, stride=w.stride, lookup=lookup)
    st = R.track_state(prev.q, prev.t, [r0] * 6)
    g = R.track_frame(vol, dev(w.depth), w.K, dev(pst), params, st)
    o = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, np.full(6, r0),
                        max_iters=w.iters, stride=w.stride, lookup=lookup, prec=orc.F32)
    assert g["iters"] == o["iters"] == w.iters
    assert g["n_points"] == o["n_points"]
    assert g["aps"][0] == o["aps"][0]
    assert np.linalg.norm(np.array(g["t"]) - o["t"]) <= 1e-4
    assert _rot_err(g["q"], o["q"]) <= 1e-4
    assert np.allclose(g["r1"], o["r1"], rtol=1e-6, atol=1e-9)
    assert abs(g["rho"] - o["rho"]) <= 1e-5


# The rescaling ablations run with the centre threshold: with the carried
# Eq. wafit threshold, a one-member APS makes the next centre that member and
# the threshold its own fitness, so particle 0 ties with the threshold and
# rounding order alone decides its membership.
@pytest.mark.parametrize("flags,early", [(1, False), (2, False), (4, False), (0, True), (8 | 4, False),
                                         (16 | 4, False)])
def test_track_frame_flags_parity(R, orc, small_gpu, flags, early):
    w, vol, psi, pst = small_gpu
    prev = w.fuse_poses[-1]
    params = R.track_params(max_iters=12, stride=w.stride, flags=flags, early_stop=early)
    st = R.track_state(prev.q, prev.t, [0.1] * 6)
    g = R.track_frame(vol, dev(w.depth), w.K, dev(pst), params, st)
    o = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, np.full(6, 0.1), max_iters=12,
                        stride=w.stride, flags=flags, early_stop=early, prec=orc.F32)
    assert g["iters"] == o["iters"]
    assert list(g["aps"]) == list(o["aps"])
    assert np.linalg.norm(np.array(g["t"]) - o["t"]) <= 1e-4
    assert _rot_err(g["q"], o["q"]) <= 1e-4


def test_track_frame_prev_depth_parity(R, orc, small_gpu):
    """pso_track_frame with the previous depth frame (holes punched into the
    last fusion depth): every O_k size, APS size and the pose equal the
    oracle's, and the option does change the overlap sets."""
    w, vol, psi, pst = small_gpu
    prev = w.fuse_poses[-1]
    rng = np.random.default_rng(11)
    prev_depth = w.fuse_depths[-1].copy()
    prev_depth[rng.random(prev_depth.shape) < 0.2] = 0.0
    prev_depth[20:70, 30:90] = 0.0
    params = R.track_params(max_iters=w.iters, stride=w.stride)
    st = R.track_state(prev.q, prev.t, [0.1] * 6)
    g = R.track_frame(vol, dev(w.depth), w.K, dev(pst), params, st, prev_depth=dev(prev_depth))
    o = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, np.full(6, 0.1),
                        max_iters=w.iters, stride=w.stride, prec=orc.F32, prev_depth=prev_depth)
    b = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, np.full(6, 0.1),
                        max_iters=w.iters, stride=w.stride, prec=orc.F32)
    assert o["n_overlap"][0] < b["n_overlap"][0]
    assert g["iters"] == o["iters"]
    assert list(g["n_overlap"]) == list(o["n_overlap"])
    assert list(g["aps"]) == list(o["aps"])
    assert np.linalg.norm(np.array(g["t"]) - o["t"]) <= 1e-4
    assert _rot_err(g["q"], o["q"]) <= 1e-4


def test_track_frame_corner_cases(R, orc, small_gpu):
    w, vol, psi, pst = small_gpu
    prev = w.fuse_poses[-1]
    params = R.track_params(max_iters=10, stride=w.stride)
    # no valid depth: status E_STATE, state untouched
    st = R.track_state(prev.q, prev.t, [0.1] * 6)
    with pytest.raises(R.RoseError) as ei:
        R.track_frame(vol, dev(np.zeros_like(w.depth)), w.K, dev(pst), params, st)
    assert ei.value.status == R.E_STATE
    assert list(st.pose.t) == list(prev.t) and st.frame == 0
    # first frame (TSDF not built): r_1 = 0.1 * 1 + 0.9 * 0.5
    st = R.track_state(prev.q, prev.t, [1.0] * 6, tsdf_built=False)
    g = R.track_frame(vol, dev(w.depth), w.K, dev(pst), params, st)
    assert np.allclose(g["r1"], 0.55) and list(st.pose.t) == list(prev.t)
    # a single particle (the centre only): every APS is empty
    st = R.track_state(prev.q, prev.t, [0.1] * 6)
    g = R.track_frame(vol, dev(w.depth), w.K, dev(pst[:1]), params, st)
    assert g["aps"] == [0] * 10 and list(st.pose.t) == list(prev.t)


@pytest.mark.parametrize("shape", [(4, 2), (8, 4), (64, 8)])
def test_track_full_size_first_iteration(R, orc, room_frame, shape):
    """Real size (512^3, 640x480, stride 4, 10240 particles): one iteration
    on the GPU equals the oracle's one iteration (APS size, centre, r_1), in
    the default launch shape and the one the bench's autotuner picks."""
    seq, vol, psi, _, _, d1 = room_frame
    pst, _ = orc.pst_sample(10240, 5600)
    prev = seq.poses[0]
    params = R.track_params(max_iters=1, stride=seq.stride)
    st = R.track_state(prev.q, prev.t, [0.55] * 6)
    try:
        R.set_fitness_shape(*shape)
        g = R.track_frame(vol, dev(d1), seq.K, dev(pst), params, st)
    finally:
        R.set_fitness_shape(4, 2)
    o = orc.track_frame(psi, seq.vox, seq.origin, d1, seq.K, pst, prev.q, prev.t, np.full(6, 0.55), max_iters=1,
                        stride=seq.stride, prec=orc.F32)
    assert g["n_points"] == o["n_points"] and g["n_overlap"][0] == o["n_overlap_last"]
    assert g["aps"][0] == o["aps"][0]
    assert np.linalg.norm(np.array(g["t"]) - o["t"]) <= 1e-4
    assert _rot_err(g["q"], o["q"]) <= 1e-4
    assert np.allclose(g["r1"], o["r1"], rtol=1e-6)


def test_track_frame_max_particles(R, orc, small_gpu):
    """The largest template the ABI accepts (ROSE_MAX_PARTICLES = 65536): one
    iteration on the small frame equals the oracle's."""
    w, vol, psi, _ = small_gpu
    pst, _ = orc.pst_sample(65536, 31)
    prev = w.fuse_poses[-1]
    params = R.track_params(max_iters=1, stride=w.stride)
    st = R.track_state(prev.q, prev.t, [0.1] * 6)
    g = R.track_frame(vol, dev(w.depth), w.K, dev(pst), params, st)
    o = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, np.full(6, 0.1), max_iters=1,
                        stride=w.stride, prec=orc.F32)
    assert g["aps"][0] == o["aps"][0] > 0
    assert np.linalg.norm(np.array(g["t"]) - o["t"]) <= 1e-4
    assert _rot_err(g["q"], o["q"]) <= 1e-4


def test_track_frame_all_points_outside(R, orc, small_gpu):
    """Degenerate frame: the camera 10 m away from the volume, so every
    point of every particle reads +1 (F = 1 for all): every APS is empty, the
    pose is kept and the axis lengths follow the empty-APS rule of Sec. 4,
    as in the oracle."""
    w, vol, psi, pst = small_gpu
    prev = w.fuse_poses[-1]
    far = np.asarray(prev.t) + np.array([10.0, 0.0, 0.0])
    params = R.track_params(max_iters=6, stride=w.stride)
    st = R.track_state(prev.q, far, [0.1] * 6)
    g = R.track_frame(vol, dev(w.depth), w.K, dev(pst), params, st)
    o = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, far, np.full(6, 0.1), max_iters=6,
                        stride=w.stride, prec=orc.F32)
    assert g["aps"] == [0] * 6 and list(o["aps"]) == [0] * 6
    assert list(st.pose.t) == list(far) and list(st.pose.q) == list(prev.q)
    assert np.allclose(g["r1"], o["r1"], rtol=1e-12, atol=0)
    assert np.allclose(g["rho_centre"], np.exp(-1.0), rtol=1e-12)


@pytest.mark.parametrize("shape", [(8, 4), (64, 8), (0, 0)])
def test_track_full_size_three_iterations(R, orc, room_frame, shape):
    """Real size in the bench's launch configurations (shape 8x4 with 16
    point slices, 64x8 with 64, the switching mode (0, 0); the particle
    schedule order): three iterations of frame 1 on the GPU equal the
    oracle's three iterations (APS sizes, overlap counts, centre, r_1)."""
    seq, vol, psi, _, _, d1 = room_frame
    pst, _ = orc.pst_sample(10240, 5600)
    prev = seq.poses[0]
    params = R.track_params(max_iters=3, stride=seq.stride)
    st = R.track_state(prev.q, prev.t, [0.55] * 6)
    try:
        R.set_fitness_shape(*shape)
        g = R.track_frame(vol, dev(d1), seq.K, dev(pst), params, st)
    finally:
        R.set_fitness_shape(4, 2)
    o = orc.track_frame(psi, seq.vox, seq.origin, d1, seq.K, pst, prev.q, prev.t, np.full(6, 0.55), max_iters=3,
                        stride=seq.stride, prec=orc.F32)
    assert g["iters"] == o["iters"] == 3
    assert list(g["aps"]) == list(o["aps"])
    assert g["n_overlap_last"] == o["n_overlap_last"]
    assert np.linalg.norm(np.array(g["t"]) - o["t"]) <= 1e-4
    assert _rot_err(g["q"], o["q"]) <= 1e-4
    assert np.allclose(g["r1"], o["r1"], rtol=1e-6)


@pytest.mark.parametrize("r0", [0.002, 0.02])
def test_track_switching_small_footprint(R, orc, room_frame, r0):
    """The switching mode with small axis lengths, where the particle-per-lane
    kernel does the work (a footprint of a few voxels), at real size: two
    iterations of frame 1 equal the oracle's (APS sizes, overlap counts,
    centre, r_1)."""
    seq, vol, psi, _, _, d1 = room_frame
    pst, _ = orc.pst_sample(10240, 5600)
    prev = seq.poses[0]
    params = R.track_params(max_iters=2, stride=seq.stride)
    st = R.track_state(prev.q, prev.t, [r0] * 6)
    try:
        R.set_fitness_shape(0, 0)
        g = R.track_frame(vol, dev(d1), seq.K, dev(pst), params, st)
    finally:
        R.set_fitness_shape(4, 2)
    o = orc.track_frame(psi, seq.vox, seq.origin, d1, seq.K, pst, prev.q, prev.t, np.full(6, r0), max_iters=2,
                        stride=seq.stride, prec=orc.F32)
    assert g["iters"] == o["iters"]
    assert list(g["aps"]) == list(o["aps"])
    assert g["n_overlap_last"] == o["n_overlap_last"]
    assert np.linalg.norm(np.array(g["t"]) - o["t"]) <= 1e-4
    assert _rot_err(g["q"], o["q"]) <= 1e-4
    assert np.allclose(g["r1"], o["r1"], rtol=1e-6)


@pytest.mark.parametrize("shape", [(4, 4), (64, 8), (0, 0)])
def test_fitness_nonfinite_and_negative_zero_transforms(R, orc, shape):
    """Particle transforms with a NaN, +inf or -inf entry put every
    evaluation outside the grid (F = 1), and a transform whose voxel x
    coordinate is exactly -0 for points at x = +0 (rotation row (-1, -0, -0),
    translation -0, origin 0) keeps those points in voxel 0 (-0 >= 0): the
    kernels' bounds test on binary32 bit patterns, after they sanitize the
    transforms, equals the oracle's float test bit for bit."""
    rng = np.random.default_rng(7)
    dims, vox, origin = (32, 24, 16), 0.04, (0.0, 0.0, 0.0)
    vol, psi = _random_volume(R, rng, dims, vox, origin, 0)
    m = 200
    pts = np.stack([np.zeros(m), rng.uniform(0.01, 0.9, m), rng.uniform(0.01, 0.6, m)], 1).astype(np.float32)
    pts[m // 2:, 0] = rng.uniform(0.0, 1.2, m - m // 2)
    T = np.zeros((5, 3, 4), np.float32)
    for i in range(5):
        T[i, :, :3] = np.eye(3)
    T[1, 0, 1] = np.nan
    T[2, 1, 3] = np.inf
    T[3, 2, 0] = -np.inf
    T[4, 0, :] = [-1.0, -0.0, -0.0, -0.0]
    T = T.reshape(5, 12)
    Fo = orc.fitness(psi, vox, np.array(origin, np.float32), pts, T.astype(np.float64), lookup=0, prec=orc.F32)
    assert Fo[1] == Fo[2] == Fo[3] == 1.0 and Fo[4] < 1.0
    try:
        vol.set_fitness_shape(*shape)
        F, _ = R.fitness_eval(vol, dev(pts), dev(T), 0)
    finally:
        vol.close()
    assert np.array_equal(host(F), Fo.astype(np.float32))
