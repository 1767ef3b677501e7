"""The order in which wavefronts take template particles (a rotation-led
Morton order, derived once per template and handle) is scheduling only: a
frame tracked with it equals, bit for bit, the same frame tracked in index
order.  A handle caches eight orders; the ninth template on a handle runs in
index order, which this test uses to get both runs through the public API."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _volume(R, w):
    vol = R.Tsdf(w.dims, w.vox, w.mu, w.origin)
    for p, d in zip(w.fuse_poses, w.fuse_depths):
        vol.integrate(dev(d), w.K, p.q, p.t)
    return vol


@pytest.mark.parametrize("shape", [(4, 2), (64, 8), (0, 0)])
@pytest.mark.parametrize("lookup", [0, 1])
def test_schedule_order_does_not_change_results(R, orc, lookup, shape):
    R.set_fitness_shape(*shape)
    try:
        _check_order(R, orc, lookup)
    finally:
        R.set_fitness_shape(4, 2)


def _check_order(R, orc, lookup):
    w = synth.small_frame()
    pst, _ = orc.pst_sample(3000, 77)
    P = dev(pst)
    depth = dev(w.depth)
    prev = w.fuse_poses[-1]
    params = R.track_params(max_iters=8, stride=w.stride, lookup=lookup)

    def run(vol):
        st = R.track_state(prev.q, prev.t, [0.3] * 6)
        r = R.track_frame(vol, depth, w.K, P, params, st)
        return r, list(st.pose.q), list(st.pose.t), list(st.r), st.rho

    ordered = _volume(R, w)
    a = run(ordered)
    plain = _volume(R, w)
    one = R.track_params(max_iters=1, stride=w.stride, lookup=lookup)
    for k in range(8):  # fill the handle's eight order slots with other (pointer, size) pairs
        st = R.track_state(prev.q, prev.t, [0.3] * 6)
        R.track_frame(plain, depth, w.K, P[: 100 + k], one, st)
    b = run(plain)
    for x, y in zip(a[1:], b[1:]):
        assert x == y
    for key in ("aps", "n_overlap", "rho_iter", "rho_centre"):
        assert a[0][key] == b[0][key], key
    ordered.close()
    plain.close()
