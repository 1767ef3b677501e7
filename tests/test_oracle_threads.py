"""The oracle's host threads (fitness over contiguous particle ranges,
fusion over z-slices) leave every result unchanged bit for bit: each
particle's and each voxel's arithmetic and point order are the same as on
one thread."""
import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def small(orc):
    w = synth.small_frame()
    psi = synth.analytic_tsdf(w.scene, w.dims, w.vox, w.origin, w.mu)
    pst, _ = orc.pst_sample(w.n_particles, w.pst_seed)
    return w, psi, pst


@pytest.mark.parametrize("lookup,prec,kahan", [(0, 1, True), (1, 1, True), (0, 0, True), (1, 0, True),
                                               (0, 1, False)])
def test_fitness_threads_bit_exact(orc, small, lookup, prec, kahan):
    w, psi, pst = small
    prev = w.fuse_poses[-1]
    pts = orc.unproject(w.depth, w.K, w.stride)
    T = orc.particle_poses(prev.q, prev.t, np.full(6, 0.05), pst[:301])
    mask = np.arange(len(pts)) % 3 != 1
    with orc.threads(1):
        a = orc.fitness(psi, w.vox, w.origin, pts, T, lookup=lookup, prec=prec, mask=mask, kahan=kahan)
    for n in (2, 7, 64, 500):  # more threads than particles included
        with orc.threads(n):
            b = orc.fitness(psi, w.vox, w.origin, pts, T, lookup=lookup, prec=prec, mask=mask, kahan=kahan)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", [1, 0])
def test_integrate_threads_bit_exact(orc, small, prec):
    w, _, _ = small
    nx, ny, nz = w.dims
    out = []
    for n in (1, 5):
        psi = np.ones((nz, ny, nx), np.float32)
        wt = np.zeros_like(psi)
        cnt = 0
        with orc.threads(n):
            for p, d in zip(w.fuse_poses, w.fuse_depths):
                cnt += orc.integrate(psi, wt, w.vox, w.origin, w.mu, d, w.K, p.q, p.t, prec=prec)
        out.append((psi, wt, cnt))
    assert out[0][2] == out[1][2] > 0
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_track_frame_threads_bit_exact(orc, small):
    w, psi, pst = small
    prev = w.fuse_poses[-1]
    res = []
    for n in (1, 6):
        with orc.threads(n):
            res.append(orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst, prev.q, prev.t, np.full(6, 0.1),
                                       max_iters=w.iters, stride=w.stride))
    a, b = res
    assert a["aps"].tolist() == b["aps"].tolist() and a["rho_iter"].tolist() == b["rho_iter"].tolist()
    assert np.array_equal(a["q"], b["q"]) and np.array_equal(a["t"], b["t"]) and np.array_equal(a["r1"], b["r1"])


def test_thread_count_is_clamped(orc):
    with orc.threads(0):
        assert orc.get_threads() == 1
    with orc.threads(10 ** 6):
        assert orc.get_threads() == 256
    assert orc.get_threads() >= 1
