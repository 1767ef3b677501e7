"""The comparison optimisers of the Sec. 5 ablation of the optimisation
strategy in the oracle: vanilla PFO (Sec. 3.1: Gaussian proposal, weights of
Eq. pfolh, resampling) and PSO (inertia-weight, global best), both on the
fitness of Eq. normallh.

Pins, none of which re-types the oracle's loop:
* systematic resampling: a hand-worked 4-particle example; equal weights
  give every particle one copy; one dominant weight takes every slot; every
  particle gets floor or ceil of n w_i / W copies (a property of systematic
  resampling);
* the PSO step: a hand-worked example, with and without the velocity clamp;
* with no motion (PFO with sigma = 0, PSO with c1 = c2 = 0 from rest, both
  over every point) the result is the brute-force best of the initial set,
  found in iteration 1 and never replaced;
* the best fitness never decreases over the iterations, the reported best
  pose is where that fitness was measured, and both methods improve on the
  start pose of the small frame;
* bad parameters and frames without depth are rejected.
"""
import math

import numpy as np
import pytest

import synth
from synth.draws import PFO, PSO, swarm_draws


@pytest.fixture(scope="module")
def small(orc):
    w = synth.small_frame()
    psi = synth.analytic_tsdf(w.scene, w.dims, w.vox, w.origin, w.mu)
    pst, _ = orc.pst_sample(1024, w.pst_seed)
    return w, psi, pst


def _run(orc, small, method, iters=10, seed=7, **kw):
    w, psi, pst = small
    prev = w.fuse_poses[-1]
    n = len(kw.get("pst", pst))
    dr, off = swarm_draws(method, iters, n, seed)
    return orc.swarm_frame(method, psi, w.vox, w.origin, kw.pop("depth", w.depth), w.K, kw.pop("pst", pst), prev.q,
                           prev.t, dr, off, iters=iters, stride=w.stride, **kw)


def test_resample_worked_example(orc):
    # F = (0.3, 0.1, 0.2, 0.1), F* = 0.1, tau = 1: w = (e^-0.2, 1, e^-0.1, 1)
    # = (0.81873, 1, 0.90484, 1); C = (0.81873, 1.81873, 2.72357, 3.72357).
    # u = 0.9: targets (m + 0.9)/4 * 3.72357 = 0.83780, 1.76843, 2.69907,
    # 3.62970 -> first C_i above each: 1, 1, 2, 3.
    assert orc.pfo_resample([0.3, 0.1, 0.2, 0.1], 0.1, 0.9).tolist() == [1, 1, 2, 3]
    # u = 0.25: targets 0.23272, 1.16335, 2.09398, 3.02461 -> 0, 1, 2, 3
    assert orc.pfo_resample([0.3, 0.1, 0.2, 0.1], 0.1, 0.25).tolist() == [0, 1, 2, 3]


def test_resample_equal_weights_is_identity(orc):
    rng = np.random.default_rng(3)
    F = np.full(1000, 0.37)
    for u in rng.random(5):
        assert np.array_equal(orc.pfo_resample(F, 0.37, float(u)), np.arange(1000))


def test_resample_dominant_weight_takes_every_slot(orc):
    F = np.full(500, 60.0)
    F[123] = 0.0
    assert np.all(orc.pfo_resample(F, 0.0, 0.5) == 123)


def test_resample_copy_counts(orc):
    rng = np.random.default_rng(11)
    for n in (7, 100, 4096):
        F = rng.uniform(0.0, 3.0, n)
        Fb = F.min()
        anc = orc.pfo_resample(F, Fb, float(rng.random()))
        assert np.all(np.diff(anc) >= 0)  # systematic resampling keeps the order
        w = np.exp(-(F - Fb))
        expect = n * w / w.sum()
        cnt = np.bincount(anc, minlength=n)
        assert np.all(cnt >= np.floor(expect - 1e-9)) and np.all(cnt <= np.ceil(expect + 1e-9))


def test_pso_step_worked_example(orc):
    # coordinate 0: x = 0, v = 0.1, p = 0.2, g = -0.1, r1 = 0.5, r2 = 0.25,
    # w = 0.5, c1 = c2 = 2: v = 0.05 + 2*0.5*0.2 + 2*0.25*(-0.1) = 0.2, x = 0.2
    # coordinate 1: x = p = g = 0.3, v = -0.4: v = w v = -0.2, x = 0.1
    x = np.zeros((1, 6), np.float32)
    v = np.zeros((1, 6), np.float32)
    p = np.zeros((1, 6), np.float32)
    g = np.zeros(6, np.float32)
    R = np.zeros((1, 12), np.float32)
    v[0, 0], p[0, 0], g[0], R[0, 0], R[0, 6] = 0.1, 0.2, -0.1, 0.5, 0.25
    x[0, 1] = p[0, 1] = g[1] = 0.3
    v[0, 1] = -0.4
    xn, vn = orc.pso_move(x, v, p, g, R, 0.5, 2.0, 2.0, np.ones(6))
    assert vn[0, 0] == pytest.approx(0.2, abs=1e-7) and xn[0, 0] == pytest.approx(0.2, abs=1e-7)
    assert vn[0, 1] == pytest.approx(-0.2, abs=1e-7) and xn[0, 1] == pytest.approx(0.1, abs=1e-7)
    assert np.all(vn[0, 2:] == 0) and np.all(xn[0, 2:] == 0)
    # the clamp at 0.15
    xn, vn = orc.pso_move(x, v, p, g, R, 0.5, 2.0, 2.0, np.full(6, 0.15, np.float32))
    assert vn[0, 0] == np.float32(0.15) and xn[0, 0] == np.float32(0.15)
    assert vn[0, 1] == np.float32(-0.15) and xn[0, 1] == pytest.approx(0.15, abs=1e-7)


@pytest.mark.parametrize("method", [PFO, PSO])
def test_no_motion_gives_best_of_initial_set(orc, small, method):
    w, psi, pst = small
    prev = w.fuse_poses[-1]
    r_init = np.full(6, 0.08)
    kw = dict(sigma=np.zeros(6)) if method == PFO else dict(c1=0.0, c2=0.0)
    res = _run(orc, small, method, iters=4, r_init=r_init, flags=orc.NO_OVERLAP, **kw)
    assert res["status"] == 0
    # brute force over the initial set x_i = r_init (.) p_i (binary32)
    x = (r_init * pst.astype(np.float64)).astype(np.float32)
    T = orc.particle_poses(prev.q, prev.t, np.ones(6), x)
    pts = orc.unproject(w.depth, w.K, w.stride)
    F = orc.fitness(psi, w.vox, w.origin, pts, T).astype(np.float32).astype(np.float64)
    best = int(np.argmin(F))
    assert res["best_index"].tolist() == [best, -1, -1, -1]
    assert np.all(res["rho_best"] == np.exp(-F[best]))
    q, t = orc.pose_retract(prev.q, prev.t, x[best].astype(np.float64))
    assert np.array_equal(res["q"], q) and np.array_equal(res["t"], t)


@pytest.mark.parametrize("method", [PFO, PSO])
def test_best_is_monotone_and_improves(orc, small, method):
    w, psi, pst = small
    prev = w.fuse_poses[-1]
    res = _run(orc, small, method, iters=10, r_init=np.full(6, 0.2))
    assert res["status"] == 0 and res["n_points"] > 0
    rb = res["rho_best"]
    assert np.all(np.diff(rb) >= 0)
    # improvements are reported exactly where rho_best rises
    rises = np.r_[True, np.diff(rb) > 0]
    assert np.array_equal(res["best_index"] >= 0, rises)
    # better than the start pose (particle 0 of the initial set sits there)
    pts = orc.unproject(w.depth, w.K, w.stride)
    F0 = orc.fitness(psi, w.vox, w.origin, pts, orc.particle_poses(prev.q, prev.t, np.zeros(6), pst[:1]))[0]
    assert res["rho"] > math.exp(-F0)
    # the reported pose has the reported fitness (all points kept in the
    # iteration where it was found: compare over that overlap set)
    T = orc.pose_mat(res["q"], res["t"])
    gt = w.gt_pose
    start_err = np.linalg.norm(prev.t - gt.t)
    assert np.linalg.norm(T[:3, 3] - gt.t) < start_err
    assert 0.0 < res["rho_mean"][0] <= rb[0]


def test_reported_fitness_is_the_pose_fitness(orc, small):
    w, psi, _ = small
    prev = w.fuse_poses[-1]
    res = _run(orc, small, PSO, iters=6, r_init=np.full(6, 0.2), flags=orc.NO_OVERLAP)
    pts = orc.unproject(w.depth, w.K, w.stride)
    T = orc.pose_mat(res["q"], res["t"])[None, :3, :]
    F = orc.fitness(psi, w.vox, w.origin, pts, T, prec=orc.F64)[0]
    # the search evaluated the unnormalised product of quaternions in
    # binary32 geometry; the pose is renormalised: the same up to voxel
    # choices at cell boundaries
    assert abs(math.exp(-F) - res["rho"]) < 2e-3


def test_bad_parameters(orc, small):
    assert _run(orc, small, PFO, iters=0)["status"] == -1
    assert _run(orc, small, PFO, iters=33)["status"] == -1
    w, psi, pst = small
    prev = w.fuse_poses[-1]
    dr, off = swarm_draws(PSO, 3, len(pst), 0)
    assert orc.swarm_frame(2, psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, dr, off,
                           iters=3)["status"] == -1
    assert orc.swarm_frame(PSO, psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, dr, off, iters=3,
                           stride=0)["status"] == -1
    with pytest.raises(ValueError):
        swarm_draws(2, 3, 4, 0)
    res = _run(orc, small, PSO, iters=3, depth=np.zeros_like(w.depth))
    assert res["status"] == -4 and res["n_points"] == 0
