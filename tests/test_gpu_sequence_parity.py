"""Whole frames and frame sequences on the GPU against the oracle, at the
real sizes: every iteration of Alg. 1 (APS sizes, overlap counts), the pose
carried from frame to frame (Sec. 4 "PST initialization": c_0 = s*^{t-1},
r_0 = r_1^{t-1}) and the fusion at each side's own tracked pose.

Bars: APS sizes and |O_k| equal in every iteration; poses within 1e-4 m and
1e-4 rad after every frame; r_1 within 1e-6 relative.  The oracle runs on
the host threads this process may use (at most 16): its threads split the
particles, never one particle's sum, so its results do not depend on them.
"""
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


@pytest.fixture(scope="module")
def nthreads(orc):
    return max(1, min(16, orc.host_threads()))


def _rot_err(qa, qb):
    Ra, Rb = synth.quat_to_mat(qa), synth.quat_to_mat(qb)
    return math.acos(float(np.clip((np.trace(Ra.T @ Rb) - 1) / 2, -1, 1)))


def _first_divergence(ga, oa):
    for k, (x, y) in enumerate(zip(ga, oa)):
        if int(x) != int(y):
            return k
    return None


def _compare(tag, g, o):
    """One tracked frame: per-iteration APS sizes and overlap counts, pose,
    r_1.  The message names the first iteration whose APS differs."""
    k = _first_divergence(g["aps"], o["aps"])
    assert g["iters"] == o["iters"], (tag, g["iters"], o["iters"])
    assert k is None, f"{tag}: APS differs first in iteration {k + 1}: gpu {g['aps']} oracle {list(o['aps'])}"
    assert list(g["n_overlap"]) == list(o["n_overlap"]), tag
    dt = float(np.linalg.norm(np.array(g["t"]) - o["t"]))
    dr = _rot_err(g["q"], o["q"])
    assert dt <= 1e-4 and dr <= 1e-4, (tag, dt, dr)
    assert np.allclose(g["r1"], o["r1"], rtol=1e-6, atol=0), tag
    return dt, dr


def _track_sequence(R, orc, seq, n_frames, n_particles, pst_seed, shape, nthreads, label):
    """Frame 0 at the given pose (the first-frame corner case of Sec. 4),
    then frames 1..n_frames-1 tracked and fused on both sides, each side
    from its own previous result."""
    depths = seq.depths(range(n_frames))
    vol = R.Tsdf(seq.dims, seq.vox, seq.mu, seq.origin)
    nx, ny, nz = seq.dims
    psi = np.ones((nz, ny, nx), np.float32)
    wt = np.zeros_like(psi)
    pst_o, _ = orc.pst_sample(n_particles, pst_seed)
    pst_g = R.pst_sample(n_particles, pst_seed)
    assert np.array_equal(pst_g.cpu().numpy(), pst_o)
    params = R.track_params(max_iters=seq.iters, stride=seq.stride)
    p0 = seq.poses[0]
    st = R.track_state(p0.q, p0.t, [1.0] * 6, tsdf_built=False)
    try:
        R.set_fitness_shape(*shape)
        R.track_frame(vol, torch.from_numpy(depths[0]).cuda(), seq.K, pst_g, params, st)
        q_o, t_o = np.array(p0.q, float), np.array(p0.t, float)
        o = orc.track_frame(psi, seq.vox, seq.origin, depths[0], seq.K, pst_o, q_o, t_o, np.ones(6),
                            tsdf_built=False, max_iters=seq.iters, stride=seq.stride, prec=orc.F32)
        r_o = o["r1"]
        assert np.allclose(list(st.r), r_o, rtol=1e-12)
        worst = (0.0, 0.0)
        for i in range(n_frames):
            if i > 0:
                g = R.track_frame(vol, torch.from_numpy(depths[i]).cuda(), seq.K, pst_g, params, st)
                with orc.threads(nthreads):
                    o = orc.track_frame(psi, seq.vox, seq.origin, depths[i], seq.K, pst_o, q_o, t_o, r_o,
                                        max_iters=seq.iters, stride=seq.stride, prec=orc.F32)
                dt, dr = _compare(f"{label} frame {i}", g, o)
                worst = (max(worst[0], dt), max(worst[1], dr))
                q_o, t_o, r_o = o["q"], o["t"], o["r1"]
            vol.integrate(torch.from_numpy(depths[i]).cuda(), seq.K, st.pose.q, st.pose.t)
            st.tsdf_built = 1
            with orc.threads(nthreads):
                orc.integrate(psi, wt, seq.vox, seq.origin, seq.mu, depths[i], seq.K, q_o, t_o, prec=orc.F32)
            print(f"[{label}] frame {i} done", flush=True)
    finally:
        R.set_fitness_shape(4, 2)
        vol.close()
    print(f"[{label}] worst pose difference over {n_frames - 1} frames: {worst[0]:.2e} m, {worst[1]:.2e} rad",
          flush=True)
    return worst


@pytest.mark.timeout(600)
def test_room_frames_switching_full(R, orc, nthreads):
    """The bench's workload and launch configuration: 512^3 at 1 cm, 640x480
    at stride 4, 10240 particles, 20 iterations, the switching mode (wide
    search footprints on the points-across kernel, narrow ones on the
    particle-per-lane kernel, chosen on the device every iteration).  Frames
    1 to 5 of the room sequence, each a full 20-iteration search, tracked
    and fused on both sides."""
    seq = synth.room_sequence(n_frames=6)
    _track_sequence(R, orc, seq, 6, 10240, 5600, (0, 0), nthreads, "room 512^3")


@pytest.mark.timeout(900)
def test_sequence_prefix_30_frames(R, orc, nthreads):
    """A 30-frame prefix of a 256^3 / 320x240 / 4096-particle sequence at
    3 m/s and 2 rad/s, tracked and fused on both sides, 20 iterations per
    frame in the switching mode."""
    seq = synth.room_sequence(scene_seed=41, traj_seed=42, noise_seed=43, n_frames=31, width=320, height=240,
                              dim=256, n_particles=4096)
    _track_sequence(R, orc, seq, 31, 4096, 5601, (0, 0), nthreads, "256^3 prefix")


CASES = [(256, 320, 4096, 1.0), (384, 640, 16384, 2.5), (512, 320, 10240, 4.0), (256, 640, 6144, 3.0)]


@pytest.fixture(scope="module")
def batch_case(R, orc, nthreads):
    """Sequences at uneven sizes (volumes 256^3 / 384^3 / 512^3, frames
    320x240 / 640x480, 4096 to 16384 particles, 1 to 4 m/s): frame 0 fused
    on both sides, and the oracle's 20-iteration search of frame 1."""
    setups, refs = [], []
    for i, (dim, width, n, speed) in enumerate(CASES):
        seq = synth.room_sequence(scene_seed=1000 + i, traj_seed=2000 + i, noise_seed=3000 + i, n_frames=3,
                                  speed=speed, ang_speed=0.67 * speed, width=width, height=width * 3 // 4, dim=dim)
        d0, d1 = seq.depths([0, 1])
        p0 = seq.poses[0]
        vol = R.Tsdf(seq.dims, seq.vox, seq.mu, seq.origin)
        vol.integrate(torch.from_numpy(d0).cuda(), seq.K, p0.q, p0.t)
        pst_o, _ = orc.pst_sample(n, 77 + i)
        setups.append((seq, vol, R.pst_sample(n, 77 + i), torch.from_numpy(d1).cuda()))
        nx, ny, nz = seq.dims
        psi = np.ones((nz, ny, nx), np.float32)
        wt = np.zeros_like(psi)
        with orc.threads(nthreads):
            orc.integrate(psi, wt, seq.vox, seq.origin, seq.mu, d0, seq.K, p0.q, p0.t, prec=orc.F32)
            del wt
            refs.append(orc.track_frame(psi, seq.vox, seq.origin, d1, seq.K, pst_o, p0.q, p0.t, np.full(6, 0.55),
                                        max_iters=20, stride=4, prec=orc.F32))
        del psi
        print(f"[batch] oracle sequence {i} done", flush=True)
    yield setups, refs
    for s in setups:
        s[1].close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("shape", [(8, 4), (64, 8), pytest.param((0, 0), marks=pytest.mark.skip(reason="a run of the batch equality test hung with the persistent kernel's switching launches (since removed, no cause found); the switching mode is covered by test_batch_step_own_launches_against_oracle"))])
def test_batch_step_against_oracle(R, batch_case, shape):
    """One batched frame step (persistent fitness launch, graph replay) of
    the uneven sequences, every sequence against the oracle's frame, in a
    points-across and the particle-per-lane launch shape."""
    setups, refs = batch_case
    params = [R.track_params(max_iters=20, stride=4) for _ in setups]
    stream = torch.cuda.Stream()
    try:
        R.set_fitness_shape(*shape)
        with torch.cuda.stream(stream):
            b = R.Batch([s[1] for s in setups], [s[0].K for s in setups], [s[2] for s in setups], params,
                        use_graph=True)
            states = (R.TrackState * len(setups))(*[R.track_state(s[0].poses[0].q, s[0].poses[0].t, [0.55] * 6)
                                                      for s in setups])
            got = b.track([s[3] for s in setups], states, stream=stream)
            b.close()
    finally:
        R.set_fitness_shape(4, 2)
    for i, (g, o) in enumerate(zip(got, refs)):
        assert g["status"] == 0
        _compare(f"batch {shape} sequence {i}", g, o)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("own_min", ["default", 60_000_000])
def test_batch_step_own_launches_against_oracle(R, batch_case, own_min):
    """The batch in the switching mode: sequences with 2^23 or more
    evaluations per iteration (here all four) take the single path's own
    switched fitness launches inside the batch's graph; with the threshold
    at 6e7 evaluations the 4800-point x 4096-particle and 4800 x 10240
    sequences share the persistent launch instead (mixed batch).  One
    batched frame step, every sequence against the oracle's frame."""
    setups, refs = batch_case
    params = [R.track_params(max_iters=20, stride=4) for _ in setups]
    stream = torch.cuda.Stream()
    try:
        R.set_fitness_shape(0, 0)
        R.set_batch_own_launch(R.BATCH_OWN_LAUNCH_DEFAULT if own_min == "default" else own_min)
        with torch.cuda.stream(stream):
            b = R.Batch([s[1] for s in setups], [s[0].K for s in setups], [s[2] for s in setups], params,
                        use_graph=True)
            states = (R.TrackState * len(setups))(*[R.track_state(s[0].poses[0].q, s[0].poses[0].t, [0.55] * 6)
                                                      for s in setups])
            got = b.track([s[3] for s in setups], states, stream=stream)
            b.close()
    finally:
        R.set_fitness_shape(4, 2)
        R.set_batch_own_launch(R.BATCH_OWN_LAUNCH_DEFAULT)
    for i, (g, o) in enumerate(zip(got, refs)):
        assert g["status"] == 0
        _compare(f"batch switching (own launches from {own_min}) sequence {i}", g, o)
