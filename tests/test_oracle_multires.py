"""Multi-resolution PST in the oracle (Sec. 4 "Multi-resolution PST": a few
(PST size, depth subsampling) pairs used in turn across the iterations).

Pins, none of which re-types the oracle's loop:
* a schedule whose levels are all the same (n, stride) is the
  single-resolution tracker, bit for bit;
* with the centre's exact fitness as the APS threshold every iteration is a
  function of (c, r) alone, so a K-iteration multi-resolution run equals K
  chained one-iteration single-resolution runs, each with its level's
  particle prefix and stride, bit for bit (the chain goes through the
  single-resolution entry, not through the schedule);
* the paper's schedule (1024, 1/8), (3072, 1/16), (10240, 1/32) -- as a
  pixel fraction, per-axis strides 3, 4, 6 -- converges on the small frame
  as the single-resolution run does;
* bad schedules are rejected, and a frame whose coarse level has no valid
  sample still runs (F = 1 there) while one with no valid sample anywhere is
  an error.
"""
import math

import numpy as np
import pytest

import synth

PAPER_LEVELS = [(1024, 3), (3072, 4), (10240, 6)]


@pytest.fixture(scope="module")
def small(orc):
    w = synth.small_frame()
    psi = synth.analytic_tsdf(w.scene, w.dims, w.vox, w.origin, w.mu)
    pst, _ = orc.pst_sample(10240, w.pst_seed)
    return w, psi, pst


def _run(orc, small, **kw):
    w, psi, pst = small
    prev = w.fuse_poses[-1]
    kw.setdefault("r_init", np.full(6, 0.1))
    r_init = kw.pop("r_init")
    return orc.track_frame(psi, w.vox, w.origin, kw.pop("depth", w.depth), w.K, kw.pop("pst", pst), prev.q, prev.t,
                           r_init, **kw)


def _pose_err(orc, res, gt):
    T = orc.pose_mat(res["q"], res["t"])
    et = np.linalg.norm(T[:3, 3] - gt.t)
    dR = T[:3, :3].T @ gt.R
    return et, math.degrees(math.acos(np.clip((np.trace(dR) - 1) / 2, -1, 1)))


@pytest.mark.parametrize("flags", [0, 4])
def test_identical_levels_equal_single_resolution(orc, small, flags):
    w, _, pst = small
    single = _run(orc, small, pst=pst[:2048], max_iters=9, stride=w.stride, flags=flags)
    multi = _run(orc, small, pst=pst[:2048], max_iters=9, stride=99, flags=flags,
                 levels=[(2048, w.stride)] * 3)
    for key in ("q", "t", "r1"):
        assert np.array_equal(single[key], multi[key]), key
    assert single["rho"] == multi["rho"] and single["iters"] == multi["iters"]
    assert np.array_equal(single["aps"], multi["aps"]) and np.array_equal(single["rho_iter"], multi["rho_iter"])


def test_schedule_equals_chained_single_iterations(orc, small):
    """Centre threshold: iteration k depends only on (c_{k-1}, r_{k-1}), the
    frame and the level, so the schedule can be replayed one iteration at a
    time through the single-resolution entry."""
    w, psi, pst = small
    levels = [(300, 4), (700, 3), (1500, 5)]
    K = 7
    multi = _run(orc, small, max_iters=K, levels=levels, flags=4)
    prev = w.fuse_poses[-1]
    q, t, r = np.array(prev.q), np.array(prev.t), np.full(6, 0.1)
    r_first = None
    for k in range(K):
        n, s = levels[k % len(levels)]
        one = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst[:n], prev.q, prev.t, r, q_init=q, t_init=t,
                              max_iters=1, stride=s, flags=4)
        assert one["aps"][0] == multi["aps"][k], k
        assert one["rho_iter"][0] == multi["rho_iter"][k], k
        q, t, r = one["q"], one["t"], one["r1"]
        if k == 0:
            r_first = r
    assert np.array_equal(q, multi["q"]) and np.array_equal(t, multi["t"])
    assert np.array_equal(r_first, multi["r1"])


def test_paper_schedule_converges(orc, small):
    w, _, _ = small
    res = _run(orc, small, max_iters=w.iters, levels=PAPER_LEVELS)
    assert res["status"] == 0 and res["iters"] == w.iters
    et, er = _pose_err(orc, res, w.gt_pose)
    assert et < 0.02 and er < 2.0  # started at 5 cm / 3 deg
    # the levels were really used: the APS of a level never exceeds its size
    for k, a in enumerate(res["aps"]):
        assert a <= PAPER_LEVELS[k % 3][0]


def test_bad_schedules_and_empty_levels(orc, small):
    w, _, pst = small
    assert _run(orc, small, levels=[(1024, 3), (20000, 4)])["status"] == -1  # more rows than the template
    assert _run(orc, small, levels=[(1024, 3), (1024, 0)])["status"] == -1
    # a sparse frame: valid depth on one pixel column not on the stride-7 grid
    d = np.zeros_like(w.depth)
    d[:, 1] = w.depth[:, 1]
    res = _run(orc, small, depth=d, max_iters=4, levels=[(512, 1), (512, 7)], flags=4)
    assert res["status"] == 0 and res["iters"] == 4
    assert res["aps"][1] == 0 and res["aps"][3] == 0  # F = 1 for every particle on the empty level
    none = _run(orc, small, depth=np.zeros_like(w.depth), levels=[(512, 1), (512, 7)])
    assert none["status"] == -4
