"""Batched tracking (many sequences in lockstep, persistent fitness launch,
HIP-graph replay): every sequence's result equals the single-sequence path
on the same inputs, graph replays equal eager launches frame after frame,
and the corner cases (first frame, empty depth) behave as in the single
path."""
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


def _volume(R, w, fmt, dims=None):
    dims = dims or w.dims
    vol = R.Tsdf(dims, w.vox, w.mu, w.origin, fmt=fmt)
    for p, d in zip(w.fuse_poses, w.fuse_depths):
        vol.integrate(torch.from_numpy(d).cuda(), w.K, p.q, p.t)
    return vol


@pytest.fixture(scope="module")
def scenes(R):
    """Three uneven sequences: different volumes (64^3 f32, 64^3 f16,
    128x64x64 f32 at a finer voxel), particle counts and strides."""
    ws = [synth.small_frame(scene_seed=2105), synth.small_frame(scene_seed=77, motion_seed=3),
          synth.small_frame(scene_seed=5, motion_seed=4, offset_m=0.03)]
    fmts = [0, 1, 0]
    ns = [1024, 3000, 512]
    strides = [3, 2, 4]
    return ws, fmts, ns, strides


def _single(R, w, fmt, n, stride, steps, lookup=0):
    vol = _volume(R, w, fmt)
    pst = R.pst_sample(n, 5600 + n)
    params = R.track_params(max_iters=w.iters, stride=stride, lookup=lookup)
    prev = w.fuse_poses[-1]
    st = R.track_state(prev.q, prev.t, [0.1] * 6)
    out = []
    for d in steps:
        out.append(R.track_frame(vol, torch.from_numpy(d).cuda(), w.K, pst, params, st))
    return out


@pytest.mark.parametrize("shape", [(4, 2), (64, 8), pytest.param((0, 0), marks=pytest.mark.skip(reason="a run of this case hung with the persistent kernel's switching launches (since removed, no cause found); the switching mode is covered by test_batch_own_launches_equal_single_path"))])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_single_path(R, scenes, use_graph, shape):
    R.set_fitness_shape(*shape)
    try:
        _batch_equals_single(R, scenes, use_graph)
    finally:
        R.set_fitness_shape(4, 2)


@pytest.mark.parametrize("own_min", [0, "default"])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_own_launches_equal_single_path(R, scenes, use_graph, own_min):
    """The switching mode: sequences with launches of their own (all of them
    at min_evals 0; at the default 2^23 only the 3000-particle one, 3000 x
    4800 evaluations, the other two sharing the persistent points-across
    launch) equal the single path bit for bit, and report which kernel did
    each iteration as it does."""
    R.set_fitness_shape(0, 0)
    R.set_batch_own_launch(0 if own_min == 0 else R.BATCH_OWN_LAUNCH_DEFAULT)
    try:
        got = _batch_equals_single(R, scenes, use_graph)
    finally:
        R.set_fitness_shape(4, 2)
        R.set_batch_own_launch(R.BATCH_OWN_LAUNCH_DEFAULT)
    ws, fmts, ns, strides = scenes
    for i, (n, s) in enumerate(zip(ns, strides)):
        evals = n * ((160 + s - 1) // s) * ((120 + s - 1) // s)
        own = own_min == 0 or evals >= R.BATCH_OWN_LAUNCH_DEFAULT
        modes, ref = got[i]["fit_mode"], got[i]["ref_fit_mode"]
        assert ref and all(m in (1, 2) for m in ref)  # the single path switched
        assert modes == (ref if own else [0] * len(modes)), (i, modes)


def _batch_equals_single(R, scenes, use_graph):
    ws, fmts, ns, strides = scenes
    # frame steps: the tracked frame, then the same frame again (a second
    # graph replay with new inputs), then a frame with no valid depth
    steps = [[w.depth, w.depth, np.zeros_like(w.depth)] for w in ws]
    ref = []
    for w, f, n, s, st_ in zip(ws, fmts, ns, strides, steps):
        ref.append(_single(R, w, f, n, s, st_[:2]))
    vols = [_volume(R, w, f) for w, f in zip(ws, fmts)]
    psts = [R.pst_sample(n, 5600 + n) for n in ns]
    params = [R.track_params(max_iters=w.iters, stride=s) for w, s in zip(ws, strides)]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = R.Batch(vols, [w.K for w in ws], psts, params, use_graph=use_graph)
        states = (R.TrackState * len(ws))(*[R.track_state(w.fuse_poses[-1].q, w.fuse_poses[-1].t, [0.1] * 6)
                                              for w in ws])
        first = []
        for k in range(3):
            depths = [torch.from_numpy(steps[i][k]).cuda() for i in range(len(ws))]
            torch.cuda.synchronize()
            _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
            got = b.track(depths, states, stream=stream)
            for i in range(len(ws)):
                if k < 2:
                    r = ref[i][k]
                    assert got[i]["status"] == 0
                    assert got[i]["aps"] == r["aps"] and got[i]["n_overlap"] == r["n_overlap"]
                    assert np.array_equal(got[i]["t"], r["t"]) and np.array_equal(got[i]["q"], r["q"])
                    assert np.array_equal(got[i]["r1"], r["r1"])
                    if k == 0:
                        first.append(dict(got[i], ref_fit_mode=r["fit_mode"]))
                else:
                    assert got[i]["status"] == R.E_STATE
                    assert np.array_equal(list(states[i].pose.t), ref[i][1]["t"])
        b.close()
    return first


def test_batch_first_frame_corner_case(R, scenes):
    ws, fmts, ns, strides = scenes
    vols = [_volume(R, w, f) for w, f in zip(ws, fmts)]
    psts = [R.pst_sample(n, 1) for n in ns]
    params = [R.track_params(max_iters=5, stride=s) for s in strides]
    b = R.Batch(vols, [w.K for w in ws], psts, params, use_graph=False)
    states = (R.TrackState * len(ws))(*[R.track_state(w.fuse_poses[-1].q, w.fuse_poses[-1].t, [1.0] * 6,
                                                      tsdf_built=(i != 1)) for i, w in enumerate(ws)])
    got = b.track([torch.from_numpy(w.depth).cuda() for w in ws], states)
    assert np.allclose(list(states[1].r), 0.55) and got[1]["iters"] == 1
    assert got[0]["iters"] == 5 and got[2]["iters"] == 5
    b.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_mixed_handle_modes_equal_single_path(R, scenes, use_graph):
    """Launch configurations set per handle: the second sequence's handle in
    the switching mode (its own launches at min_evals 0), the others on the
    process-wide fixed shape (4, 2) in the persistent launch.  Every
    sequence equals the single path run on a handle configured the same
    way, and reports the kernel of each iteration as that path does."""
    ws, fmts, ns, strides = scenes
    R.set_batch_own_launch(0)
    try:
        ref, vols = [], []
        for i, (w, f, n, s) in enumerate(zip(ws, fmts, ns, strides)):
            v = _volume(R, w, f)
            if i == 1:
                v.set_fitness_shape(0, 0)
            st = R.track_state(w.fuse_poses[-1].q, w.fuse_poses[-1].t, [0.1] * 6)
            ref.append(R.track_frame(v, torch.from_numpy(w.depth).cuda(), w.K, R.pst_sample(n, 5600 + n),
                                     R.track_params(max_iters=w.iters, stride=s), st))
            v.close()
            v = _volume(R, w, f)
            if i == 1:
                v.set_fitness_shape(0, 0)
            vols.append(v)
        psts = [R.pst_sample(n, 5600 + n) for n in ns]
        params = [R.track_params(max_iters=w.iters, stride=s) for w, s in zip(ws, strides)]
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            b = R.Batch(vols, [w.K for w in ws], psts, params, use_graph=use_graph)
            states = (R.TrackState * len(ws))(*[R.track_state(w.fuse_poses[-1].q, w.fuse_poses[-1].t, [0.1] * 6)
                                                  for w in ws])
            got = b.track([torch.from_numpy(w.depth).cuda() for w in ws], states, stream=stream)
            b.close()
        for i, r in enumerate(ref):
            assert got[i]["status"] == 0
            assert got[i]["aps"] == r["aps"] and got[i]["n_overlap"] == r["n_overlap"], i
            assert np.array_equal(got[i]["t"], r["t"]) and np.array_equal(got[i]["q"], r["q"]), i
            assert np.array_equal(got[i]["r1"], r["r1"]), i
            assert got[i]["fit_mode"] == (r["fit_mode"] if i == 1 else [0] * len(got[i]["fit_mode"])), i
        assert all(m in (1, 2) for m in ref[1]["fit_mode"])
        for v in vols:
            v.close()
    finally:
        R.set_batch_own_launch(R.BATCH_OWN_LAUNCH_DEFAULT)
