"""Pins of the oracle's PST update (Alg. 1; Eqs. ebs, rsdir, rsinter,
momentum, wafit; Sec. 4 corner cases) and of the whole per-frame loop."""
import math

import numpy as np
import pytest

import synth


def _pst(rows):
    return np.asarray(rows, dtype=np.float32)


def test_worked_three_particle_example(orc):
    """Hand-worked example.  F = (ln 2, ln 4/3, 0) gives rho = (1/2, 3/4, 1).
    APS = {1, 2}; w = (1/4, 1/2), normalised (1/3, 2/3).
    With r = 1 and p1 = (0,0,0, 3/8,0,0), p2 = (0,0,0, 0,3/4,0):
      u* = (0,0,0, 1/8, 1/2, 0),  rho~ = (1/4*3/4 + 1/2*1)/(3/4) = 11/12,
      ||v|| = sqrt(17/64),  rhat = (1/12) |v|/||v|| + 1e-3,
      r = 0.1 * 1 + 0.9 * rhat,  centre moves by (1/8, 1/2, 0) in its frame."""
    pst = _pst([[0] * 6, [0, 0, 0, 0.375, 0, 0], [0, 0, 0, 0, 0.75, 0]])
    F = [math.log(2.0), math.log(4.0 / 3.0), 0.0]
    qc = np.array([1.0, 0, 0, 0])
    tc = np.array([1.0, 2.0, 3.0])
    out = orc.pst_update(F, pst, np.ones(6), qc, tc)
    assert out["aps"] == 2
    assert out["u_star"] == pytest.approx([0, 0, 0, 0.125, 0.5, 0], abs=1e-15)
    assert out["rho_tilde"] == pytest.approx(11 / 12, abs=1e-12)
    nv = math.sqrt(17 / 64)
    rhat = np.array([0, 0, 0, 0.125 / nv, 0.5 / nv, 0]) / 12 + 1e-3
    assert out["r"] == pytest.approx(0.1 + 0.9 * rhat, abs=1e-14)
    assert out["t"] == pytest.approx([1.125, 2.5, 3.0], abs=1e-15)
    assert out["q"] == pytest.approx([1, 0, 0, 0], abs=1e-15)


def test_single_member_aps_moves_to_that_particle(orc):
    pst, _ = orc.pst_sample(64, 9)
    rng = np.random.default_rng(0)
    qc = synth.mat_to_quat(synth.axis_angle([0.3, -1, 0.2], 0.7))
    tc = rng.standard_normal(3)
    r = rng.uniform(0.05, 0.5, 6)
    F = np.full(64, 0.5)
    F[17] = 0.2
    out = orc.pst_update(F, pst, r, qc, tc)
    assert out["aps"] == 1
    u = r * pst[17].astype(np.float64)
    assert np.allclose(out["u_star"], u, atol=1e-15)
    assert out["rho_tilde"] == pytest.approx(math.exp(-0.2), rel=1e-14)
    T = orc.particle_poses(qc, tc, r, pst[17:18])[0]
    assert np.allclose(synth.quat_to_mat(out["q"]), T[:, :3], atol=1e-12)
    assert np.allclose(out["t"], T[:, 3], atol=1e-12)


def test_symmetric_aps_gives_zero_step_and_isotropic_scale(orc):
    p = [0.1, -0.2, 0.05, 0.3, 0.0, -0.1]
    pst = _pst([[0] * 6, p, [-v for v in p]])
    F = [1.0, 0.5, 0.5]
    out = orc.pst_update(F, pst, np.ones(6), [1, 0, 0, 0], [0, 0, 0])
    assert out["aps"] == 2
    assert np.allclose(out["u_star"], 0, atol=1e-17)
    rt = math.exp(-0.5)
    assert out["r"] == pytest.approx(0.1 + 0.9 * ((1 - rt) / math.sqrt(6) + 1e-3), rel=1e-12)


def test_empty_aps_corner_case(orc):
    pst, _ = orc.pst_sample(32, 3)
    F = np.linspace(0.3, 0.9, 32)  # row 0 is the best
    r = np.full(6, 0.2)
    out = orc.pst_update(F, pst, r, [1, 0, 0, 0], [0.5, 0, 0])
    assert out["aps"] == 0
    rho0 = math.exp(-0.3)
    assert out["r"] == pytest.approx(0.1 * 0.2 + 0.9 * 2 * (1 - rho0) / math.sqrt(6), rel=1e-13)
    assert np.array_equal(out["t"], [0.5, 0, 0]) and np.array_equal(out["q"], [1, 0, 0, 0])


def test_tsdf_not_built_corner_case(orc):
    pst, _ = orc.pst_sample(8, 3)
    out = orc.pst_update(np.zeros(8), pst, np.ones(6), [1, 0, 0, 0], [0, 0, 0], tsdf_built=False)
    assert out["r"] == pytest.approx(np.full(6, 0.55), abs=1e-15)
    assert out["rho_tilde"] == 0.5


def test_update_is_permutation_invariant(orc):
    rng = np.random.default_rng(1)
    pst, _ = orc.pst_sample(200, 4)
    F = rng.uniform(0.1, 0.4, 200)
    F[0] = 0.25
    a = orc.pst_update(F, pst, np.full(6, 0.3), [1, 0, 0, 0], [0, 0, 0])
    perm = np.concatenate([[0], 1 + rng.permutation(199)])
    b = orc.pst_update(F[perm], pst[perm], np.full(6, 0.3), [1, 0, 0, 0], [0, 0, 0])
    assert a["aps"] == b["aps"]
    assert np.allclose(a["u_star"], b["u_star"], atol=1e-15)
    assert np.allclose(a["r"], b["r"], atol=1e-15)


# ------------------------------------------------------------ whole frame
@pytest.fixture(scope="module")
def small(orc):
    w = synth.small_frame()
    psi = synth.analytic_tsdf(w.scene, w.dims, w.vox, w.origin, w.mu)
    pst, _ = orc.pst_sample(w.n_particles, w.pst_seed)
    return w, psi, pst


def _pose_err(orc, res, gt):
    T = orc.pose_mat(res["q"], res["t"])
    et = np.linalg.norm(T[:3, 3] - gt.t)
    dR = T[:3, :3].T @ gt.R
    er = math.degrees(math.acos(np.clip((np.trace(dR) - 1) / 2, -1, 1)))
    return et, er


@pytest.mark.parametrize("lookup", [0, 1])
def test_track_small_frame_converges(orc, small, lookup):
    w, psi, pst = small
    prev = w.fuse_poses[-1]
    res = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, np.full(6, 0.1),
                          max_iters=w.iters, stride=w.stride, lookup=lookup)
    assert res["status"] == 0 and res["iters"] == w.iters
    et, er = _pose_err(orc, res, w.gt_pose)
    assert et < 0.02 and er < 2.0  # started at 5 cm / 3 deg
    pts = orc.unproject(w.depth, w.K, w.stride)
    Tf = orc.pose_mat(res["q"], res["t"])[:3]
    F_found = orc.fitness(psi, w.vox, w.origin, pts, Tf[None], lookup=lookup)[0]
    F_start = orc.fitness(psi, w.vox, w.origin, pts, prev.as_3x4()[None], lookup=lookup)[0]
    assert F_found < 0.2 * F_start


def test_track_early_stop_and_first_frame(orc, small):
    w, psi, pst = small
    prev = w.fuse_poses[-1]
    res = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, np.full(6, 0.1),
                          max_iters=20, stride=w.stride, early_stop=True)
    assert 1 <= res["iters"] <= 20
    if res["iters"] < 20:
        a = res["aps"]
        assert (len(a) >= 2 and a[-1] == 0 and a[-2] == 0) or a[-1] > 0
    r0 = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, np.ones(6), tsdf_built=False)
    assert r0["iters"] == 1 and np.allclose(r0["r1"], 0.55)
    assert np.array_equal(r0["q"], prev.q) and np.array_equal(r0["t"], prev.t)


def test_track_no_points_is_an_error(orc, small):
    w, psi, pst = small
    prev = w.fuse_poses[-1]
    res = orc.track_frame(psi, w.vox, w.origin, np.zeros_like(w.depth), w.K, pst, prev.q, prev.t, np.full(6, 0.1))
    assert res["status"] == -4 and np.array_equal(res["t"], prev.t)


def test_brute_force_grid_agrees_with_search(orc):
    """Tiny scene: a 16^3 TSDF of a room corner and ~60 points.  A 7^6 grid
    (1 cm, 0.01 quaternion steps) around the true pose has its argmin at
    the true pose, and PST search from a 2 cm / 2 degree offset reaches an
    objective no worse than the grid's second-best value within the paper's
    20 iterations (both APS threshold readings)."""
    scene = synth.Scene(np.array([-0.2, -0.2, -0.2]), np.array([0.15, 0.17, 0.16]),
                        spheres=[synth.Sphere(np.array([0.05, -0.05, 0.1]), 0.06)])
    dims, vox, mu = (16, 16, 16), 0.025, 0.075
    origin = np.full(3, -0.2)
    psi = synth.analytic_tsdf(scene, dims, vox, origin, mu)
    K = synth.Intrinsics.centred(40, 30, 30.0)
    gt = synth.Pose(synth.look_rotation([1, 1.2, 0.9]), np.array([-0.05, -0.05, -0.06]))
    depth = synth.render_depth(scene, K, gt)
    pts = orc.unproject(depth, K, 4, 0)
    assert 40 <= len(pts) <= 80
    steps = np.arange(-3, 4)
    grid = np.stack(np.meshgrid(*([steps] * 6), indexing="ij"), -1).reshape(-1, 6).astype(np.float64)
    u = grid * np.array([0.01, 0.01, 0.01, 0.01, 0.01, 0.01])
    qg = gt.q
    T = orc.particle_poses(qg, gt.t, np.ones(6), u.astype(np.float32))
    F = orc.fitness(psi, vox, origin, pts, T, lookup=1, prec=0)
    best = int(np.argmin(F))
    assert np.all(grid[best] == 0)
    pst, _ = orc.pst_sample(1024, 5600)
    start = synth.Pose(synth.axis_angle([0, 1, 0], math.radians(2.0)) @ gt.R, gt.t + np.array([0.02, 0, 0]))
    second = np.partition(F, 1)[1]
    # both readings of the APS threshold within the paper's 20-iteration cap
    # (Sec. 4 "Convergence criteria")
    for flags, iters in ((0, 20), (orc.CENTRE_THRESHOLD, 20)):
        res = orc.track_frame(psi, vox, origin, depth, K, pst, start.q, start.t, np.full(6, 0.1), max_iters=iters,
                              stride=4, lookup=1, flags=flags)
        Tf = orc.pose_mat(res["q"], res["t"])[:3]
        Ff = orc.fitness(psi, vox, origin, pts, Tf[None], lookup=1, prec=0)[0]
        assert Ff <= second


@pytest.mark.parametrize("flag", ["iso", "aniso"])
def test_rescaling_ablation_worked_example(orc, flag):
    """The worked example above with one part of Eq. rsinter switched off:
    isotropic only -> rhat_d = (1 - 11/12) / sqrt6 + 1e-3 on every axis;
    anisotropic only -> rhat = |v| / ||v|| + 1e-3.  The centre moves as in
    the full scheme; the empty-APS branch is unaffected."""
    pst = _pst([[0] * 6, [0, 0, 0, 0.375, 0, 0], [0, 0, 0, 0, 0.75, 0]])
    F = [math.log(2.0), math.log(4.0 / 3.0), 0.0]
    f = orc.ISO_ONLY if flag == "iso" else orc.ANISO_ONLY
    out = orc.pst_update(F, pst, np.ones(6), [1, 0, 0, 0], [1.0, 2.0, 3.0], flags=f)
    nv = math.sqrt(17 / 64)
    if flag == "iso":
        rhat = np.full(6, (1 / 12) / math.sqrt(6)) + 1e-3
    else:
        rhat = np.array([0, 0, 0, 0.125 / nv, 0.5 / nv, 0]) + 1e-3
    assert out["aps"] == 2
    assert out["r"] == pytest.approx(0.1 + 0.9 * rhat, abs=1e-14)
    assert out["t"] == pytest.approx([1.125, 2.5, 3.0], abs=1e-15)
    empty = orc.pst_update([0.3, 0.5, 0.9], pst, np.full(6, 0.2), [1, 0, 0, 0], [0, 0, 0], flags=f)
    assert empty["aps"] == 0
    assert empty["r"] == pytest.approx(0.02 + 0.9 * 2 * (1 - math.exp(-0.3)) / math.sqrt(6), rel=1e-13)


# ---------------------------------------------- the APS threshold, replayed
def _replay(orc, psi, w, pst, r0, lookup, iters, rule):
    """Alg. 1 for one frame, one iteration at a time, through the oracle's
    single-iteration update (pst_update), with the APS threshold chosen here:
      carry  -- Sec. 4: the fitness of s*_k is never evaluated and Eq. wafit
                stands in for it, so the threshold of iteration k >= 2 is
                rho~ of the last iteration whose APS was non-empty; at k = 1
                (s*_0 = c_0) it is the centre's own fitness (template row 0);
      centre -- the centre's exact fitness at every k;
      reset  -- a slip: back to the centre's fitness after an empty APS."""
    pts = orc.unproject(w.depth, w.K, w.stride, orc.F32)
    prev = w.fuse_poses[-1]
    Tprev = orc.pose_mat(prev.q, prev.t)
    qc, tc, r = np.array(prev.q, float), np.array(prev.t, float), np.full(6, float(r0))
    thr, r1, rho_last, empty_before = None, None, None, False
    aps, rts = [], []
    for k in range(1, iters + 1):
        mask = orc.overlap(pts, orc.pose_mat(qc, tc), Tprev, w.K, orc.F32)
        T = orc.particle_poses(qc, tc, r, pst)
        F = orc.fitness(psi, w.vox, w.origin, pts, T, lookup=lookup, prec=orc.F32, mask=mask)
        F = F.astype(np.float32).astype(np.float64)  # the tracker keeps F in binary32
        centre = math.exp(-F[0])
        if rule == "carry":
            t_k = centre if k == 1 else thr
        elif rule == "centre":
            t_k = centre
        else:
            t_k = centre if (k == 1 or empty_before) else thr
        out = orc.pst_update(F, pst, r, qc, tc, rho_thr=t_k)
        thr = out["rho_tilde"] if out["aps"] > 0 else t_k
        empty_before = out["aps"] == 0
        aps.append(out["aps"])
        rts.append(out["rho_tilde"])
        if out["aps"] > 0 or rho_last is None:
            rho_last = out["rho_tilde"]
        qc, tc, r = out["q"], out["t"], out["r"]
        if k == 1:
            r1 = r.copy()
    return dict(aps=aps, rho_iter=rts, q=qc, t=tc, r1=r1, rho=rho_last)


@pytest.mark.parametrize("lookup,r0", [(0, 0.55), (1, 0.1)])
def test_threshold_carry_replayed_exactly(orc, lookup, r0):
    """orc_track_frame equals, bit for bit, an independent replay of its
    loop whose APS threshold follows the Eq. wafit reading; the two inputs
    exercise an empty APS before any non-empty one (r0 = 0.55: the
    threshold stays the centre's fitness) and an empty APS after a
    one-member APS followed by a non-empty one (r0 = 0.1, trilinear: the
    carried rho~ survives the empty step).  The slips "reset to the centre
    after an empty APS" and "centre every k" give different results on the
    second input, so the replay tells them apart."""
    w = synth.small_frame()
    psi = synth.analytic_tsdf(w.scene, w.dims, w.vox, w.origin, w.mu)
    pst, _ = orc.pst_sample(w.n_particles, w.pst_seed)
    prev = w.fuse_poses[-1]
    iters = 20
    res = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, np.full(6, r0),
                          max_iters=iters, stride=w.stride, lookup=lookup)
    rep = _replay(orc, psi, w, pst, r0, lookup, iters, "carry")
    assert res["aps"].tolist() == rep["aps"]
    assert res["rho_iter"].tolist() == rep["rho_iter"]
    assert np.array_equal(res["q"], rep["q"]) and np.array_equal(res["t"], rep["t"])
    assert np.array_equal(res["r1"], rep["r1"]) and res["rho"] == rep["rho"]
    a = rep["aps"]
    first_full = next(k for k, n in enumerate(a) if n > 0)
    if r0 == 0.55:
        assert a[0] == 0 and first_full == 1  # empty first, then a non-empty step
    else:
        # a one-member APS, then an empty one, then a non-empty one
        assert any(a[k] == 1 and a[k + 1] == 0 and a[k + 2] > 0 for k in range(len(a) - 2))
        for rule in ("reset", "centre"):
            alt = _replay(orc, psi, w, pst, r0, lookup, iters, rule)
            assert alt["aps"] != rep["aps"] or not np.array_equal(alt["t"], rep["t"])
