"""Volumes of 4 GB and more: the fitness kernel switches to 64-bit byte
offsets.  A 1032 x 1024 x 1024 binary32 volume (4.3 GB of psi) is filled with
+1 and random values in a block near its far z end, so that the gathered
voxels lie beyond the first 4 GB of the buffer; fitness of poses that map the
points into that block equals the oracle's (relative 1e-5), for both lookups,
and the import round-trips."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

DIMS = (1032, 1024, 1024)  # nx, ny, nz: 1.08e9 voxels, > 2^30 (binary32 bytes > 2^32)
VOX = 0.01


@pytest.fixture(scope="module")
def wide(orc):
    from paper_2105_05600_amd import rose
    nx, ny, nz = DIMS
    rng = np.random.default_rng(77)
    psi = np.ones((nz, ny, nx), np.float32)
    block = psi[960:1024, 448:576, 448:576]
    block[...] = rng.uniform(-1, 1, block.shape).astype(np.float32)
    vol = rose.Tsdf(DIMS, VOX, 3 * VOX, (0.0, 0.0, 0.0))
    vol.load(torch.from_numpy(psi.reshape(-1)).cuda())
    torch.cuda.synchronize()
    return rose, vol, psi


def test_wide_volume_is_wide(wide):
    _, vol, _ = wide
    assert vol.psi.numel() * 4 >= 2 ** 32


@pytest.mark.parametrize("lookup", [0, 1])
def test_wide_fitness_parity(orc, wide, lookup):
    rose, vol, psi = wide
    rng = np.random.default_rng(5 + lookup)
    # points around the random block's centre (5.12, 5.12, 9.92) m, camera frame = world frame
    pts = (np.array([5.12, 5.12, 9.92]) + rng.uniform(-0.5, 0.5, (3000, 3)) * [1.2, 1.2, 0.5]).astype(np.float32)
    n = 37
    T = np.zeros((n, 3, 4), np.float32)
    for i in range(n):
        a = rng.standard_normal(3)
        a = a / np.linalg.norm(a) * rng.uniform(0, 0.002)
        K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
        T[i, :, :3] = np.eye(3) + K  # first-order rotation (the oracle takes T as given)
        T[i, :, 3] = rng.uniform(-0.02, 0.02, 3)
    F, _ = rose.fitness_eval(vol, torch.from_numpy(pts).cuda(), torch.from_numpy(T).cuda(), lookup)
    F = F.cpu().numpy()
    Fo = orc.fitness(psi, VOX, np.zeros(3, np.float32), pts, T.astype(np.float64), lookup=lookup, prec=orc.F32)
    assert np.all(Fo < 0.9)  # the points really land in the random block
    assert np.max(np.abs(F - Fo) / np.abs(Fo)) <= 1e-5


def test_wide_export_round_trip(wide):
    _, vol, psi = wide
    g, _ = vol.export()
    g = g.cpu().numpy()
    assert np.array_equal(g[960:1024, 448:576, 448:576].view(np.uint32),
                          psi[960:1024, 448:576, 448:576].view(np.uint32))
    assert np.all(g[:960:97] == 1.0)
