"""Pins of the oracle's pose algebra: the 6D chart of Sec. 3.3 (quaternion
imaginary part + translation) and the MovePST composition, checked against
Rodrigues' axis-angle formula (an independent closed form)."""
import math

import numpy as np

import synth


def _rodrigues_from_u(u):
    v = np.asarray(u[:3], dtype=np.float64)
    s = np.linalg.norm(v)
    if s == 0:
        return np.eye(3)
    theta = 2 * math.asin(min(s, 1.0))
    return synth.axis_angle(v / s, theta)


def _random_rotation(rng):
    return synth.axis_angle(rng.standard_normal(3), rng.uniform(0, math.pi))


def test_chart_identity(orc):
    q, t = orc.chart_delta(np.zeros(6))
    assert np.array_equal(q, [1, 0, 0, 0]) and np.array_equal(t, [0, 0, 0])


def test_chart_is_half_angle(orc):
    # u = (sin(theta/2) a, 0) is the rotation by theta about a
    rng = np.random.default_rng(3)
    for _ in range(20):
        a = rng.standard_normal(3)
        a /= np.linalg.norm(a)
        th = rng.uniform(0, 3.0)
        u = np.concatenate([math.sin(th / 2) * a, rng.standard_normal(3)])
        q, t = orc.chart_delta(u)
        R = synth.quat_to_mat(q)
        assert np.allclose(R, synth.axis_angle(a, th), atol=1e-12)
        assert np.array_equal(t, u[3:])


def test_particle_pose_against_rodrigues(orc):
    rng = np.random.default_rng(4)
    pst, _ = orc.pst_sample(50, 77)
    for _ in range(5):
        Rc = _random_rotation(rng)
        tc = rng.standard_normal(3)
        qc = synth.mat_to_quat(Rc)
        r = rng.uniform(0.01, 1.0, 6)
        T = orc.particle_poses(qc, tc, r, pst)
        for i in range(len(pst)):
            u = r * pst[i].astype(np.float64)
            Rd = _rodrigues_from_u(u)
            R_exp = Rc @ Rd
            t_exp = Rc @ u[3:] + tc
            assert np.allclose(T[i, :, :3], R_exp, atol=1e-12)
            assert np.allclose(T[i, :, 3], t_exp, atol=1e-12)
            # a proper rotation
            assert np.allclose(T[i, :, :3] @ T[i, :, :3].T, np.eye(3), atol=1e-12)
        # row 0 is the centre itself
        assert np.allclose(T[0, :, :3], Rc, atol=1e-12) and np.allclose(T[0, :, 3], tc, atol=1e-15)


def test_retract_matches_particle_pose(orc):
    """Moving the centre to u* and reading the particle at u* agree."""
    rng = np.random.default_rng(5)
    Rc = _random_rotation(rng)
    qc = synth.mat_to_quat(Rc)
    tc = rng.standard_normal(3)
    u = rng.uniform(-0.3, 0.3, 6)
    q, t = orc.pose_retract(qc, tc, u)
    assert q[0] >= 0 and abs(np.linalg.norm(q) - 1) < 1e-15
    R_exp = Rc @ _rodrigues_from_u(u)
    assert np.allclose(synth.quat_to_mat(q), R_exp, atol=1e-12)
    assert np.allclose(t, Rc @ u[3:] + tc, atol=1e-12)


def test_chart_saturates_outside_unit_ball(orc):
    q, _ = orc.chart_delta(np.array([2.0, 0, 0, 0, 0, 0]))
    assert np.allclose(q, [0, 1, 0, 0])  # rotation by pi about x
