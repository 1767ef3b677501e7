"""The largest frame the ABI accepts (ROSE_MAX_IMAGE_PIXELS = 4096 x 4096):
unprojection at stride 1 (16.7 million samples, with holes) and the overlap
mask of all its points are bit-exact against the oracle, and the fitness of
16 poses over the stride-2 points (4.2 million) is within 1e-5."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

W = H = 4096


@pytest.fixture(scope="module")
def R():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2105_05600_amd import rose
    return rose


@pytest.fixture(scope="module")
def frame():
    K = synth.Intrinsics.centred(W, H, 3000.0)
    u = np.arange(W, dtype=np.float32)
    v = np.arange(H, dtype=np.float32)
    depth = (1.5 + 0.5 * v[:, None] / H + 0.25 * u[None, :] / W).astype(np.float32)
    depth[::7, ::5] = 0.0  # missing measurements
    return K, depth


def test_max_image_unproject_and_overlap(R, orc, frame):
    K, depth = frame
    g = R.depth_unproject(torch.from_numpy(depth).cuda(), K, 1)
    o = orc.unproject(depth, K, 1)
    assert g.shape[0] == o.shape[0] == W * H - ((H + 6) // 7) * ((W + 4) // 5)
    gh = g.cpu().numpy()
    assert np.array_equal(gh.view(np.uint32), o.view(np.uint32))
    qc = synth.mat_to_quat(synth.axis_angle(np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8]),
                                            np.deg2rad(4.0)))
    tc = np.array([0.12, -0.05, -0.3])  # towards the scene: about 30 % of the points leave the image
    prev = (np.array([1.0, 0.0, 0.0, 0.0]), np.zeros(3))
    mg = R.overlap_mask(g, (qc, tc), prev, K).cpu().numpy()
    mo = orc.overlap(o, orc.pose_mat(qc, tc), orc.pose_mat(*prev), K)
    assert 0 < mo.sum() < len(mo)  # the band at the border is cut
    assert np.array_equal(mg, mo)


def test_max_image_fitness(R, orc, frame):
    K, depth = frame
    dims, vox, origin = (128, 128, 128), 0.02, np.array([-1.28, -1.28, 0.5], np.float32)
    rng = np.random.default_rng(4096)
    psi = rng.uniform(-1, 1, (dims[2], dims[1], dims[0])).astype(np.float32)
    vol = R.Tsdf(dims, vox, 3 * vox, origin)
    vol.load(torch.from_numpy(psi.reshape(-1)).cuda())
    pts = orc.unproject(depth, K, 2)
    T = np.zeros((16, 3, 4), np.float32)
    for i in range(16):
        a = rng.standard_normal(3) * 0.01
        Kx = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
        T[i, :, :3] = np.eye(3) + Kx
        T[i, :, 3] = rng.uniform(-0.03, 0.03, 3)
    F, _ = R.fitness_eval(vol, torch.from_numpy(pts).cuda(), torch.from_numpy(T).cuda())
    Fo = orc.fitness(psi, vox, origin, pts, T.astype(np.float64), prec=orc.F32)
    assert np.max(np.abs(F.cpu().numpy() - Fo) / np.abs(Fo)) <= 1e-5
    vol.close()
