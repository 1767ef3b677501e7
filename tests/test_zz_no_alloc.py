"""fitness_eval_noalloc (no device allocation: the library's fixed scratch)
against fitness_eval on the same inputs, through the C ABI: two calls in a
row on one handle, the second with fewer points and particles (the scratch
keeps the first call's contents), then a third at the size limits of the
point count; every result equal to fitness_eval's bit for bit (NEAREST and
TRILINEAR: same kernels, same exact sums)."""
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


def _volume(R, rng, dims, vox, origin):
    nx, ny, nz = dims
    psi = rng.uniform(-1, 1, (nz, ny, nx)).astype(np.float32)
    psi[rng.random((nz, ny, nx)) < 0.2] = 1.0
    vol = R.Tsdf(dims, vox, 3 * vox, origin)
    vol.load(torch.from_numpy(psi.ravel()).cuda())
    return vol


def _poses(rng, n):
    T = np.zeros((n, 3, 4), np.float32)
    for i in range(n):
        T[i, :, :3] = synth.axis_angle(rng.standard_normal(3), rng.uniform(0, 0.3))
        T[i, :, 3] = rng.uniform(-0.1, 0.1, 3)
    return torch.from_numpy(T.reshape(n, 12)).cuda()


@pytest.mark.parametrize("lookup", [0, 1])
def test_noalloc_equals_fitness_eval(R, lookup):
    rng = np.random.default_rng(77 + lookup)
    vol = _volume(R, rng, (32, 24, 16), 0.04, (-0.64, -0.48, -0.32))
    cases = [(3001, 130), (65, 9), (R._lib.fitness_eval_noalloc_max_points(), 3)]
    try:
        for m, n in cases:
            pts = torch.from_numpy(rng.uniform(-0.7, 0.7, (m, 3)).astype(np.float32)).cuda()
            T = _poses(rng, n)
            F0, rho0 = R.fitness_eval(vol, pts, T, lookup)
            F = torch.full((n,), -1.0, device="cuda")
            rho = torch.full((n,), -1.0, device="cuda")
            R.fitness_eval_noalloc(vol, pts, T, F, rho, lookup)
            torch.cuda.synchronize()
            assert torch.equal(F, F0) and torch.equal(rho, rho0), (m, n)
            assert bool(((F >= 0) & (F <= 1)).all())
    finally:
        vol.close()


def test_noalloc_rejects_oversize(R):
    rng = np.random.default_rng(5)
    vol = _volume(R, rng, (16, 16, 16), 0.05, (-0.4, -0.4, -0.4))
    m = R._lib.fitness_eval_noalloc_max_points() + 1
    pts = torch.zeros((m, 3), device="cuda")
    T = _poses(rng, 2)
    F = torch.empty(2, device="cuda")
    rho = torch.empty(2, device="cuda")
    try:
        with pytest.raises(R.RoseError):
            R.fitness_eval_noalloc(vol, pts, T, F, rho)
    finally:
        vol.close()
