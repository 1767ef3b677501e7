"""Handle-level behaviour of the C ABI on the GPU: per-handle launch
configuration (two handles with different shapes in one process), no device
memory left behind by create / track / destroy cycles, and stream ordering
of pso_track_frame on a non-default stream."""
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


def _volume(R, w, shape=None):
    vol = R.Tsdf(w.dims, w.vox, w.mu, w.origin)
    for p, d in zip(w.fuse_poses, w.fuse_depths):
        vol.integrate(torch.from_numpy(d).cuda(), w.K, p.q, p.t)
    if shape is not None:
        vol.set_fitness_shape(*shape)
    return vol


def _rot_err(qa, qb):
    Ra, Rb = synth.quat_to_mat(qa), synth.quat_to_mat(qb)
    return math.acos(float(np.clip((np.trace(Ra.T @ Rb) - 1) / 2, -1, 1)))


def _track(R, vol, w, pst, iters=None):
    prev = w.fuse_poses[-1]
    params = R.track_params(max_iters=iters or w.iters, stride=w.stride)
    st = R.track_state(prev.q, prev.t, [0.1] * 6)
    return R.track_frame(vol, torch.from_numpy(w.depth).cuda(), w.K, pst, params, st)


def test_per_handle_shapes_against_oracle(R, orc):
    """Three handles over the same fused frame, each with its own launch
    configuration (points-across 4x8, one particle per lane, switching with
    a 4x4 wide side), interleaved in one process while the process-wide
    default is something else: every frame equals the oracle's (APS sizes,
    pose within 1e-4 m / 1e-4 rad), and a handle reset to (-1, -1) follows
    the process-wide default again."""
    w = synth.small_frame()
    nx, ny, nz = w.dims
    psi = np.ones((nz, ny, nx), np.float32)
    wt = np.zeros_like(psi)
    for p, d in zip(w.fuse_poses, w.fuse_depths):
        orc.integrate(psi, wt, w.vox, w.origin, w.mu, d, w.K, p.q, p.t, prec=orc.F32)
    pst_o, _ = orc.pst_sample(w.n_particles, w.pst_seed)
    pst = R.pst_sample(w.n_particles, w.pst_seed)
    prev = w.fuse_poses[-1]
    o = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst_o, prev.q, prev.t, np.full(6, 0.1),
                        max_iters=w.iters, stride=w.stride, prec=orc.F32)
    vols = [_volume(R, w, (4, 8)), _volume(R, w, (64, 8)), _volume(R, w)]
    vols[2].set_fitness_switch(16.0, 3.0, wide=(4, 4))
    vols[2].set_fitness_shape(0, 0)
    try:
        R.set_fitness_shape(8, 2)
        for _round in range(2):
            for v in vols:
                g = _track(R, v, w, pst)
                assert g["aps"] == list(o["aps"])
                assert np.linalg.norm(np.array(g["t"]) - o["t"]) <= 1e-4 and _rot_err(g["q"], o["q"]) <= 1e-4
        vols[0].set_fitness_shape(-1, -1)
        g = _track(R, vols[0], w, pst)
        assert g["aps"] == list(o["aps"])
    finally:
        R.set_fitness_shape(4, 2)
        for v in vols:
            v.close()


def test_per_handle_shape_rejects_bad_values(R):
    w = synth.small_frame()
    vol = R.Tsdf(w.dims, w.vox, w.mu, w.origin)
    try:
        with pytest.raises(R.RoseError):
            vol.set_fitness_shape(3, 3)
        with pytest.raises(R.RoseError):
            vol.set_fitness_switch(16.0, 3.0, wide=(64, 8))
        with pytest.raises(R.RoseError):
            vol.set_fitness_switch(-1.0, 3.0)
    finally:
        vol.close()


def test_create_destroy_cycles_release_device_memory(R):
    """Handles grow device scratch on demand (points, partial sums, device
    state, schedule orders); tsdf_destroy frees all of it: after a warm
    cycle, ten create / integrate / track / fitness_eval / destroy cycles
    leave the free device memory unchanged (hipMemGetInfo)."""
    w = synth.small_frame()
    pst = R.pst_sample(w.n_particles, w.pst_seed)
    pts = torch.rand((500, 3), device="cuda")
    T = torch.eye(3, 4, device="cuda").repeat(300, 1, 1).reshape(300, 12).contiguous()

    def cycle():
        vol = _volume(R, w)
        _track(R, vol, w, pst, iters=3)
        R.fitness_eval(vol, pts, T, 0)
        torch.cuda.synchronize()
        vol.close()
        torch.cuda.synchronize()

    cycle()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(10):
        cycle()
    torch.cuda.empty_cache()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0 - (2 << 20), (free0, free1)


def test_track_frame_on_non_default_stream(R):
    """pso_track_frame enqueues on the caller's stream: a depth frame that is
    produced on that stream right before the call (behind a long kernel, no
    host synchronisation) is the one tracked, and the result equals the same
    frame tracked on the default stream."""
    w = synth.small_frame()
    pst = R.pst_sample(w.n_particles, w.pst_seed)
    vol_a = _volume(R, w)
    vol_b = _volume(R, w)
    ref = _track(R, vol_a, w, pst)
    src = torch.from_numpy(w.depth).cuda()
    big = torch.rand((4096, 4096), device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    prev = w.fuse_poses[-1]
    params = R.track_params(max_iters=w.iters, stride=w.stride)
    st = R.track_state(prev.q, prev.t, [0.1] * 6)
    with torch.cuda.stream(s):
        for _ in range(4):
            big = big @ big * 1e-3  # keeps the stream busy
        depth = torch.zeros_like(src)
        depth.copy_(src + 0.0 * big[0, 0])
        got = R.track_frame(vol_b, depth, w.K, pst, params, st, stream=s)
    assert got["aps"] == ref["aps"]
    assert got["t"] == ref["t"] and got["q"] == ref["q"]
    vol_a.close()
    vol_b.close()


def test_template_order_cache_forget(R):
    """The schedule-order cache (speed only): a template tracked on a handle
    is cached once; a template rewritten in place keeps the cached order and
    still gives the results of a fresh handle (the order changes no result);
    tsdf_forget_templates empties the cache and the next frame caches again."""
    w = synth.small_frame()
    vol = _volume(R, w)
    fresh = _volume(R, w)
    try:
        pst = R.pst_sample(w.n_particles, w.pst_seed)
        a = _track(R, vol, w, pst)
        assert vol.template_orders() == 1
        # new rows written into the same buffer: the cached order is stale
        pst.copy_(R.pst_sample(w.n_particles, w.pst_seed + 1))
        b = _track(R, vol, w, pst)
        assert vol.template_orders() == 1
        c = _track(R, fresh, w, pst)
        assert b["aps"] == c["aps"] and b["t"] == c["t"] and b["q"] == c["q"]
        assert a["aps"] != b["aps"] or a["t"] != b["t"]  # a different template tracks differently
        vol.forget_templates()
        assert vol.template_orders() == 0
        d = _track(R, vol, w, pst)
        assert vol.template_orders() == 1
        assert d["aps"] == c["aps"] and d["t"] == c["t"] and d["q"] == c["q"]
    finally:
        vol.close()
        fresh.close()
