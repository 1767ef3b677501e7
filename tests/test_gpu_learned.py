"""GPU path of the learned-proposal inputs and network against the oracle:
raycast (binary64 geometry on both sides), residual features, the BF16
matrix-core GEMM, network forward / gradients (against the oracle with the
same BF16 operand rounding: relative L2 <= 2e-4 / 5e-4, loss 1e-4; against
the binary64 oracle: 1e-2) and the Adam step."""
import numpy as np
import pytest
import torch

import synth
import synth.mlp_init as mi
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    assert torch.cuda.is_available()
    from paper_2105_05600_amd import rose
    return rose


def _bf16(a):
    """Round float32 to bfloat16 (nearest even), returned as float64."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("M,N,K,ta,tb", [(32, 32, 8, False, False), (64, 64, 32, False, False),
                                         (70, 45, 37, False, False), (33, 130, 300, True, False),
                                         (200, 12, 256, False, True), (5, 256, 1216, False, False)])
def test_gemm_bf16_matches_exact_products(R, M, N, K, ta, tb):
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
    B = rng.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
    At = torch.from_numpy(A).cuda()
    Bt = torch.from_numpy(B).cuda()
    At = At.t() if ta else At
    Bt = Bt.t() if tb else Bt
    C = R.gemm_bf16(At, Bt).cpu().numpy().astype(np.float64)
    Ab = _bf16(A.T if ta else A)
    Bb = _bf16(B.T if tb else B)
    ref = Ab @ Bb
    scale = np.abs(Ab) @ np.abs(Bb)
    assert np.all(np.abs(C - ref) <= 1e-5 * scale + 1e-30)


@pytest.fixture(scope="module")
def small_vol(R, orc):
    """The small frame's volume fused on the GPU (vol) and by the oracle
    (psi, the oracle's input)."""
    w = synth.small_frame()
    vol = R.Tsdf(w.dims, w.vox, w.mu, w.origin)
    nx, ny, nz = w.dims
    psi = np.ones((nz, ny, nx), np.float32)
    wt = np.zeros_like(psi)
    for p, d in zip(w.fuse_poses, w.fuse_depths):
        vol.integrate(torch.from_numpy(d).cuda(), w.K, p.q, p.t)
        orc.integrate(psi, wt, w.vox, w.origin, w.mu, d, w.K, p.q, p.t, prec=orc.F32)
    return w, vol, psi


def test_raycast_parity(R, orc, small_vol):
    w, vol, psi = small_vol
    K = synth.Intrinsics(40, 30, w.K.fx / 4, w.K.fy / 4, (w.K.cx + 0.5) / 4 - 0.5, (w.K.cy + 0.5) / 4 - 0.5)
    pose = w.fuse_poses[-1]
    step = float(np.float32(w.vox)) / 2
    g = R.raycast(vol, pose.q, pose.t, K, near=0.05, far=2.0, step=step).cpu().numpy()
    o = orc.raycast(psi, w.vox, w.origin, pose.q, pose.t, K, near=0.05, far=2.0, step=step)
    assert (o > 0).mean() > 0.9
    assert np.array_equal(g > 0, o > 0)
    assert np.abs(g - o).max() <= 1e-6


def test_features_parity(R, orc, small_vol):
    w, vol, psi = small_vol
    K = synth.Intrinsics(40, 30, w.K.fx / 4, w.K.fy / 4, (w.K.cx + 0.5) / 4 - 0.5, (w.K.cy + 0.5) / 4 - 0.5)
    pose = w.fuse_poses[-1]
    rend = R.raycast(vol, pose.q, pose.t, K, near=0.05, far=2.0)
    depth = w.depth.copy()
    depth[::7, ::5] = 0
    vel = [0.01, -0.02, 0.003, 0.05, 0.0, -0.1]
    f = R.proposal_features(torch.from_numpy(depth).cuda(), w.K, rend, K, 4, vel, 1216).cpu().numpy()
    o = orc.proposal_features(depth, rend.cpu().numpy(), 4, vel, 1216)
    assert np.array_equal(f, o)


def _cos_rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300)
    rel = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300)
    return cos, rel


@pytest.fixture(scope="module")
def net(R):
    m = R.Mlp(1216, 256, 12, max_batch=512)
    p = mi.init_params(5)
    rng = np.random.default_rng(9)
    p["W3"] = (rng.standard_normal(p["W3"].shape) * 0.05).astype(np.float32)
    X = np.zeros((300, 1216), np.float32)
    X[:, :1206] = rng.standard_normal((300, 1206)).astype(np.float32) * 0.2
    Y = (rng.standard_normal((300, 6)) * 0.05).astype(np.float32)
    return m, p, X, Y


def test_mlp_forward_vs_oracle(R, net):
    """Against the oracle with the same BF16 operand rounding the matrix
    cores apply (binary64 products): only the binary32 accumulation (over
    K up to 1216; the single GEMM stays within 1e-5 of sum |a b|) and the
    binary32 elementwise arithmetic differ, rel. L2 <= 2e-4 (observed
    7e-5); against the plain binary64 network the BF16 operands cost ~1 %."""
    m, p, X, _ = net
    out = m.forward(m.pack(p), torch.from_numpy(X).cuda()).cpu().numpy()
    p64 = {k: v.astype(np.float64) for k, v in p.items()}
    ref, _ = omlp.forward(p64, X, bf16=True)
    cos, rel = _cos_rel(out, ref)
    print(f"forward vs the BF16-operand oracle: cos {cos:.9f}, rel {rel:.3e}")
    assert cos >= 0.9999999 and rel <= 2e-4
    ref64, _ = omlp.forward(p64, X)
    cos, rel = _cos_rel(out, ref64)
    assert cos >= 0.999 and rel <= 1e-2


def test_mlp_gradients_vs_oracle(R, net):
    m, p, X, Y = net
    P = m.pack(p)
    G = torch.zeros_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    m.loss_grad(P, torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), G, loss)
    gl = float(loss.item())
    p64 = {k: v.astype(np.float64) for k, v in p.items()}
    ol, og = omlp.loss_and_grads(p64, X, Y, bf16=True)
    print(f"loss {gl:.9g} vs the BF16-operand oracle {ol:.9g}")
    assert abs(gl - ol) <= 1e-4 * abs(ol)
    gg = m.unpack(G.cpu())
    for k in omlp.NAMES:
        cos, rel = _cos_rel(gg[k].numpy(), og[k])
        print(f"grad {k}: cos {cos:.9f}, rel {rel:.3e}")
        # gradient sums over the batch cancel heavily, which raises the
        # relative error of the binary32 accumulation (observed <= 1.5e-4)
        assert cos >= 0.9999999 and rel <= 5e-4, (k, cos, rel)
    ol64, og64 = omlp.loss_and_grads(p64, X, Y)
    assert abs(gl - ol64) <= 2e-2 * abs(ol64)  # the BF16 operands themselves: ~1 %


def test_adam_vs_oracle(R):
    rng = np.random.default_rng(1)
    n = 1000
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m0 = (rng.standard_normal(n) * 0.1).astype(np.float32)
    v0 = np.abs(rng.standard_normal(n) * 0.1).astype(np.float32)
    P, Gt, M, V = (torch.from_numpy(a.copy()).cuda() for a in (p, g, m0, v0))
    R.Mlp.adam(P, Gt, M, V, step=3, lr=1e-3)
    po = {k: p.astype(np.float64).copy() for k in ["x"]}
    mo = {"x": m0.astype(np.float64)}
    vo = {"x": v0.astype(np.float64)}
    omlp.adam_step(po, {"x": g.astype(np.float64)}, mo, vo, 3, lr=1e-3)
    assert np.allclose(P.cpu().numpy(), po["x"], rtol=0, atol=2e-6)
    assert np.allclose(M.cpu().numpy(), mo["x"], rtol=1e-6, atol=1e-7)
    assert np.allclose(V.cpu().numpy(), vo["x"], rtol=1e-6, atol=1e-7)
