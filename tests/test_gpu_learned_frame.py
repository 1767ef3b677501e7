"""The learned frame as a whole (pso_track_frame_learned) against an oracle
composition of the same steps, each an oracle function: raycast of the model
at the previous pose through the low-resolution camera, residual features,
the network forward (BF16 operands), the proposal (chart retraction of the
previous pose by mu, axis lengths kappa exp(l) clamped to [r_min, r_max]),
the search from that proposal with the small template and the learned
iteration count, and the rule that keeps it when its final fitness is at
least the previous frame's minus delta, else tracks the frame again with
plain PST from the unchanged state (also when the network output is not
finite).

The network's weights are zero and its first two biases zero, so both
sides' outputs are exactly its last bias (GELU(0) = 0 on both): the
composition is then compared without the last-bit difference of the two
forward passes, which would move the search centre by ~1e-7 and can flip a
near-tied APS decision.  The forward pass itself, the raycast and the
features are compared with the oracle in test_gpu_learned.py.  Tolerances
are those of the plain frame: 1e-4 m / 1e-4 rad, r_1 to 1e-6 relative,
rho to 1e-5, and equal fallback decisions."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

N_SMALL, SMALL_ITERS, RHO_PREV = 512, 5, 0.3
# mu (rad, m) and the log axis lengths, all exact in binary32
MU = [0.001953125, -0.0009765625, 0.00048828125, 0.00390625, -0.001953125, 0.0029296875]
LOGR = [-3.5, -3.5, -3.5, -3.0, -3.0, -3.0]


@pytest.fixture(scope="module")
def R():
    assert torch.cuda.is_available()
    from paper_2105_05600_amd import rose
    return rose


@pytest.fixture(scope="module")
def frame(R, orc):
    w = synth.small_frame()
    vol = R.Tsdf(w.dims, w.vox, w.mu, w.origin)
    nx, ny, nz = w.dims
    psi = np.ones((nz, ny, nx), np.float32)
    wt = np.zeros_like(psi)
    for p, d in zip(w.fuse_poses, w.fuse_depths):
        vol.integrate(torch.from_numpy(d).cuda(), w.K, p.q, p.t)
        orc.integrate(psi, wt, w.vox, w.origin, w.mu, d, w.K, p.q, p.t, prec=orc.F32)
    yield w, vol, psi
    vol.close()


def _params(b3):
    z = lambda *s: np.zeros(s, np.float32)  # noqa: E731
    return {"W1": z(1216, 256), "b1": z(256), "W2": z(256, 256), "b2": z(256), "W3": z(256, 12),
            "b3": np.asarray(b3, np.float32)}


def _low_camera(K, scale, w, h):
    f32 = np.float32
    return synth.Intrinsics(width=w, height=h, fx=float(f32(K.fx) / f32(scale)), fy=float(f32(K.fy) / f32(scale)),
                            cx=float((f32(K.cx) + f32(0.5)) / f32(scale) - f32(0.5)),
                            cy=float((f32(K.cy) + f32(0.5)) / f32(scale) - f32(0.5)))


def _oracle_learned(orc, w, psi, params, pst_small, pst_plain, lp, prev, r_prev, velocity):
    """Returns (result, fallback) of the learned frame, every step by the oracle."""
    K_low = _low_camera(w.K, lp.scale, lp.low_w, lp.low_h)
    render = orc.raycast(psi, w.vox, w.origin, prev.q, prev.t, K_low, near=lp.near_m, far=lp.far_m, step=lp.step_m)
    X = orc.proposal_features(w.depth, render, lp.scale, velocity, lp.feature_dim)
    out = omlp.forward(params, X[None, :], bf16=True)[0][0]
    plain = dict(max_iters=w.iters, stride=w.stride, prec=orc.F32)
    if np.all(np.isfinite(out)):
        qc, tc = orc.pose_retract(prev.q, prev.t, out[:6])
        r0 = np.minimum(lp.r_max, np.maximum(lp.r_min, lp.kappa * orc.exp_rho(out[6:])))
        trial = orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst_small, prev.q, prev.t, r0, q_init=qc,
                                t_init=tc, max_iters=SMALL_ITERS, stride=w.stride, prec=orc.F32)
        if trial["status"] == 0 and trial["rho"] >= RHO_PREV - lp.delta:
            return trial, False
    return orc.track_frame(psi, w.vox, w.origin, w.depth, w.K, pst_plain, prev.q, prev.t, r_prev, **plain), True


def _rot_err(qa, qb):
    qa, qb = np.asarray(qa, np.float64), np.asarray(qb, np.float64)
    return 2.0 * np.arccos(min(1.0, abs(float(qa @ qb)) / (np.linalg.norm(qa) * np.linalg.norm(qb))))


@pytest.mark.parametrize("case,shape", [("keep", (4, 2)), ("keep", (0, 0)), ("regress", (4, 2)),
                                        ("nonfinite", (4, 2))])
def test_learned_frame_against_oracle_composition(R, orc, frame, case, shape):
    w, vol, psi = frame
    prev = w.fuse_poses[-1]
    r_prev = np.full(6, 0.1)
    velocity = [0.01, -0.02, 0.005, 0.03, 0.0, -0.01]
    b3 = MU + LOGR
    if case == "nonfinite":
        b3 = [float("nan")] + b3[1:]
    # "regress": no trial can come within -delta = 2 of the previous fitness
    lp = R.learned_params(scale=4, low_w=40, low_h=30, feature_dim=1216, kappa=2.0, r_min=1e-3, r_max=1.0,
                          delta=(-2.0 if case == "regress" else 0.5), near=0.05, far=2.0, step=0.005,
                          iters=SMALL_ITERS)
    params = _params(b3)
    pst_small_o, _ = orc.pst_sample(N_SMALL, 91)
    pst_plain_o, _ = orc.pst_sample(w.n_particles, w.pst_seed)
    o, o_fb = _oracle_learned(orc, w, psi, params, pst_small_o, pst_plain_o, lp, prev, r_prev, velocity)

    net = R.Mlp(1216, 256, 12, max_batch=64)
    work = torch.zeros(40 * 30 + 1216 + 12, device="cuda")
    st = R.track_state(prev.q, prev.t, r_prev)
    st.rho = RHO_PREV
    tp = R.track_params(max_iters=w.iters, stride=w.stride)
    vol.set_fitness_shape(*shape)
    try:
        g = R.track_frame_learned(vol, torch.from_numpy(w.depth).cuda(), w.K, R.pst_sample(N_SMALL, 91),
                                  R.pst_sample(w.n_particles, w.pst_seed), net, net.pack(params), work, velocity,
                                  tp, lp, st)
    finally:
        vol.set_fitness_shape(-1, -1)
        net.close()
    assert g["fallback"] == o_fb == (case != "keep"), (g["fallback"], o_fb)
    assert g["iters"] == o["iters"] == (SMALL_ITERS if case == "keep" else w.iters)
    assert g["n_points"] == o["n_points"]
    assert g["aps"][0] == o["aps"][0]
    assert np.linalg.norm(np.array(g["t"]) - o["t"]) <= 1e-4
    assert _rot_err(g["q"], o["q"]) <= 1e-4
    assert np.allclose(g["r1"], o["r1"], rtol=1e-6, atol=1e-9)
    assert abs(g["rho"] - o["rho"]) <= 1e-5
