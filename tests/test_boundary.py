"""The C-ABI library loads, exports every declared symbol, and validates
arguments on the host before touching the device (no GPU needed)."""
import ctypes as C

import pytest


@pytest.fixture(scope="module")
def R():
    from paper_2105_05600_amd import rose
    return rose


def test_every_declared_symbol_is_exported(R):
    names = R.header_functions()
    expected = {"tsdf_create", "tsdf_integrate", "pst_sample", "pso_track_frame", "fitness_eval", "tsdf_destroy",
                "tsdf_bytes", "tsdf_export", "tsdf_import", "rose_last_error"}
    assert expected <= set(names)
    missing = [n for n in names if not hasattr(R._lib, n)]
    assert missing == []


def test_version(R):
    assert "gfx950" in R.version()


def test_tsdf_bytes(R):
    lib = R._lib
    assert lib.tsdf_bytes(64, 64, 64, R.F32, 0) == 64**3 * 4
    assert lib.tsdf_bytes(64, 64, 64, R.F32, 1) == 64**3 * 4
    assert lib.tsdf_bytes(512, 512, 512, R.F16, 0) == 512**3 * 2
    assert lib.tsdf_bytes(512, 512, 512, R.SN16, 1) == 512**3 * 2
    for bad in [(0, 8, 8), (12, 8, 8), (8, 8, 4096), (-8, 8, 8)]:
        assert lib.tsdf_bytes(*bad, R.F32, 0) == 0
    assert lib.tsdf_bytes(8, 8, 8, 7, 0) == 0
    assert lib.tsdf_bytes(8, 8, 8, R.F32, 2) == 0
    assert lib.tsdf_bytes(2048, 2048, 1024, R.F32, 0) == 0  # above 2^31 voxels


def test_host_side_argument_errors(R):
    lib = R._lib
    assert lib.pst_sample(0, 1, C.c_void_p(16), None) == R.E_ARG
    assert b"out of" in lib.rose_last_error()
    assert lib.pst_sample(R_MAX := 65537, 1, C.c_void_p(16), None) == R.E_ARG
    assert lib.pst_sample(8, 1, None, None) == R.E_ARG
    h = C.c_void_p()
    org = (C.c_float * 3)(0, 0, 0)
    assert lib.tsdf_create(12, 8, 8, 0.01, 0.03, org, R.F32, 128.0, C.c_void_p(16), C.c_void_p(16), None,
                           C.byref(h)) == R.E_SHAPE
    assert lib.tsdf_create(8, 8, 8, -0.01, 0.03, org, R.F32, 128.0, C.c_void_p(16), C.c_void_p(16), None,
                           C.byref(h)) == R.E_ARG
    assert lib.tsdf_create(8, 8, 8, 0.01, 0.03, org, R.F32, 128.0, None, C.c_void_p(16), None,
                           C.byref(h)) == R.E_ARG
    assert lib.tsdf_destroy(None) == R.OK
    cam = R.Camera(100, 100, 10, 10, 0, 20)
    assert lib.depth_unproject(C.c_void_p(16), C.byref(cam), 2, 0, C.c_void_p(16), C.c_void_p(16), None) == R.E_SHAPE
    cam = R.Camera(100, 100, 10, 10, 4096, 4097)  # one row above ROSE_MAX_IMAGE_PIXELS
    assert lib.depth_unproject(C.c_void_p(16), C.byref(cam), 2, 0, C.c_void_p(16), C.c_void_p(16), None) == R.E_SHAPE
    cam = R.Camera(100, 100, 10, 10, 20, 20)
    assert lib.depth_unproject(C.c_void_p(16), C.byref(cam), 0, 0, C.c_void_p(16), C.c_void_p(16), None) == R.E_ARG
    assert lib.depth_unproject(C.c_void_p(16), C.byref(cam), 2, 5, C.c_void_p(16), C.c_void_p(16), None) == R.E_ARG
    assert lib.rose_fitness_set_shape(3, 3) == R.E_UNSUPPORTED
    assert lib.fitness_eval(None, None, 0, None, 1, 0, None, None, None) == R.E_ARG
    v16 = C.c_void_p(16)
    big = lib.fitness_eval_noalloc_max_points() + 1
    assert lib.fitness_eval_noalloc_max_points() == 131072
    assert lib.fitness_eval_noalloc(None, v16, 10, v16, 1, 0, v16, None, None) == R.E_ARG
    assert lib.fitness_eval_noalloc(v16, v16, big, v16, 1, 0, v16, None, None) == R.E_ARG
    assert b"out of [0, 131072]" in lib.rose_last_error()
    assert lib.fitness_eval_noalloc(v16, v16, 10, v16, 0, 0, v16, None, None) == R.E_ARG
    assert lib.fitness_eval_noalloc(v16, v16, 10, v16, 1, 7, v16, None, None) == R.E_ARG
    params = R.track_params(max_iters=0)
    st = R.track_state([1, 0, 0, 0], [0, 0, 0], [0.1] * 6)
    assert lib.pso_track_frame(C.c_void_p(16), C.c_void_p(16), None, C.byref(cam), C.c_void_p(16), 16,
                               C.byref(params), None, None, C.byref(st), None, None) == R.E_ARG
    params = R.track_params(max_iters=10)
    assert lib.pso_track_frame(C.c_void_p(16), C.c_void_p(16), None, C.byref(cam), C.c_void_p(16), 0,
                               C.byref(params), None, None, C.byref(st), None, None) == R.E_ARG
    params = R.track_params(levels=[(8, 2), (16, 3)])
    assert lib.pso_track_frame(C.c_void_p(16), C.c_void_p(16), None, C.byref(cam), C.c_void_p(16), 12,
                               C.byref(params), None, None, C.byref(st), None, None) == R.E_ARG  # level larger than the template
    assert b"level 1" in lib.rose_last_error()
    params = R.track_params(flags=R.FLAG_ISO_ONLY | R.FLAG_ANISO_ONLY)
    assert lib.pso_track_frame(C.c_void_p(16), C.c_void_p(16), None, C.byref(cam), C.c_void_p(16), 16,
                               C.byref(params), None, None, C.byref(st), None, None) == R.E_ARG
    params = R.track_params(levels=[(8, 2), (16, 3)])
    params.levels = R.MAX_LEVELS + 1
    assert lib.pso_track_frame(C.c_void_p(16), C.c_void_p(16), None, C.byref(cam), C.c_void_p(16), 16,
                               C.byref(params), None, None, C.byref(st), None, None) == R.E_ARG
    assert lib.rose_profile_read(None) == R.E_ARG
    assert lib.tsdf_forget_templates(None) == R.E_ARG
    assert lib.tsdf_template_orders(None) == 0
    assert lib.rose_gather_peak(C.c_void_p(16), 1 << 20, 3000, 8, 1, 1, C.c_void_p(16), None) == R.E_ARG
    assert lib.rose_gather_peak(C.c_void_p(16), 1 << 10, 4096, 8, 1, 1, C.c_void_p(16), None) == R.E_SHAPE
    assert lib.rose_gather_peak(C.c_void_p(16), 1 << 20, 64, 12, 1, 1, C.c_void_p(16), None) == R.E_ARG
    assert lib.rose_gather_peak_loads_per_lane() == 8
    assert lib.rose_l2_read_peak(C.c_void_p(16), 1 << 20, 3000, 8, 1, C.c_void_p(16), None) == R.E_ARG
    assert lib.rose_l2_read_peak(C.c_void_p(16), 1 << 10, 4096, 8, 1, C.c_void_p(16), None) == R.E_SHAPE
    assert lib.rose_l2_read_peak(C.c_void_p(16), 1 << 20, 4096, 12, 1, C.c_void_p(16), None) == R.E_ARG
    assert lib.rose_l2_read_peak(C.c_void_p(16), 1 << 20, 4096, 8, 0, C.c_void_p(16), None) == R.E_ARG
    v = C.c_void_p(16)
    assert lib.pst_poisson(0, 1, 0.3, 100, v, v, v, None) == R.E_ARG
    assert lib.pst_poisson(8, 1, 2.5, 100, v, v, v, None) == R.E_ARG
    assert lib.pst_poisson(8, 1, 0.3, -1, v, v, v, None) == R.E_ARG
    assert lib.pst_poisson(8, 1, 0.3, 100, None, v, v, None) == R.E_ARG
    lp = R.learned_params()
    assert lib.pso_batch_track_learned(None, None, None, None, None, None, C.byref(lp), None, None, None, None, None,
                                       None, None) == R.E_ARG
    lp.iters = 99
    assert lib.pso_track_frame_learned(v, v, C.byref(cam), v, 16, v, 16, v, v, v, (C.c_double * 6)(),
                                       C.byref(R.track_params()), C.byref(lp), C.byref(st), None, None,
                                       None) == R.E_ARG


def test_swarm_argument_errors(R):
    """vanilla_pfo_track_frame / plain_pso_track_frame validate everything on
    the host; with tsdf_built = 0 they keep the pose without touching the
    device or the handle."""
    lib = R._lib
    fake = C.c_void_p(16)  # never dereferenced on these paths
    cam = R.Camera(100, 100, 10, 10, 20, 20)
    st = R.track_state([1, 0, 0, 0], [0.1, 0.2, 0.3], [1.0] * 6)
    stats = R.SwarmStats()

    def pfo(params, n=8, normals=fake, offsets=fake, h=fake, state=st):
        return lib.vanilla_pfo_track_frame(h, fake, C.byref(cam), fake, n, C.byref(params), normals, offsets,
                                           C.byref(state), C.byref(stats), None)

    def pso(params, n=8, uniforms=fake):
        return lib.plain_pso_track_frame(fake, fake, C.byref(cam), fake, n, C.byref(params), uniforms, C.byref(st),
                                         C.byref(stats), None)

    ok = R.swarm_params(iters=5)
    assert pfo(ok, h=None) == R.E_ARG
    assert pfo(ok, n=0) == R.E_ARG and pfo(ok, n=65537) == R.E_ARG
    assert pfo(R.swarm_params(iters=0)) == R.E_ARG and pfo(R.swarm_params(iters=33)) == R.E_ARG
    assert pfo(R.swarm_params(stride=0)) == R.E_ARG
    assert pfo(R.swarm_params(lookup=2)) == R.E_ARG
    assert pfo(R.swarm_params(flags=R.FLAG_CENTRE_THRESHOLD)) == R.E_ARG
    assert b"only ROSE_FLAG_NO_OVERLAP" in lib.rose_last_error()
    assert pfo(R.swarm_params(tau=0.0)) == R.E_ARG
    assert pfo(R.swarm_params(r_init=[0.1] * 5 + [-0.1])) == R.E_ARG
    assert pfo(R.swarm_params(sigma=[float("nan")] * 6)) == R.E_ARG
    assert pso(R.swarm_params(vmax=[-1.0] * 6)) == R.E_ARG
    assert pso(R.swarm_params(c1=float("inf"))) == R.E_ARG
    assert pfo(ok, normals=None) == R.E_ARG and pfo(ok, offsets=None) == R.E_ARG
    assert pso(ok, uniforms=None) == R.E_ARG
    # one iteration needs no draws
    cold = R.track_state([1, 0, 0, 0], [0.1, 0.2, 0.3], [1.0] * 6, tsdf_built=False)
    assert pfo(R.swarm_params(iters=1), normals=None, offsets=None, state=cold) == R.OK
    assert list(cold.pose.t) == [0.1, 0.2, 0.3] and cold.frame == 1 and stats.iters == 0


def test_profile_launch_log_host_side(R):
    """With nothing timed, the per-launch fitness log is empty (no device
    call needed); NULL count pointers are rejected."""
    R.profile_reset()
    assert len(R.profile_fitness_launches()) == 0
    assert R._lib.rose_profile_fitness_launches(None, 0, None) == R.E_ARG


def test_fitness_shapes_host_side(R):
    """rose_fitness_set_shape accepts the compiled shapes and (0, 0) (the
    switching mode) and refuses everything else with ROSE_E_UNSUPPORTED;
    rose_fitness_set_switch checks its range and restores its defaults with
    a zero threshold; no device call is made."""
    lib = R._lib
    try:
        for p, u in [(2, 4), (4, 2), (4, 4), (8, 2), (8, 4), (64, 4), (64, 8), (64, 16), (0, 0)]:
            assert lib.rose_fitness_set_shape(p, u) == R.OK, (p, u)
        for p, u in [(64, 2), (64, 32), (16, 4), (1, 1), (0, 4), (-1, -1)]:
            assert lib.rose_fitness_set_shape(p, u) == R.E_UNSUPPORTED, (p, u)
        for thr, z in [(-1.0, 3.0), (8.0, -0.5), (2e6, 3.0)]:
            assert lib.rose_fitness_set_switch(thr, z) == R.E_ARG, (thr, z)
        R.set_fitness_switch(8.0, 3.0)
        assert lib.rose_fitness_set_switch(0.0, 0.0) == R.OK  # the defaults
    finally:
        assert lib.rose_fitness_set_shape(4, 2) == R.OK


def test_batch_own_launch_setting_host_side(R):
    """rose_batch_set_own_launch takes any min_evals >= 0 and refuses a
    negative one; no device call is made."""
    lib = R._lib
    try:
        assert lib.rose_batch_set_own_launch(-1) == R.E_ARG
        assert b"negative" in lib.rose_last_error()
        for v in (0, 1, 1 << 40):
            assert lib.rose_batch_set_own_launch(v) == R.OK
    finally:
        R.set_batch_own_launch(R.BATCH_OWN_LAUNCH_DEFAULT)
