"""CPU oracle for PST pose search against a TSDF (ROSEFusion, Sec. 3-4).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
baseline of the benchmark may import this package.  The product library
never does; it shares no code with this package.

The arithmetic lives in ``rose_oracle.c`` (plain single-threaded C, built
with gcc, no FMA contraction); this module builds it and exposes numpy-level
wrappers via ctypes.

Parity status per function (what pins it, tests/test_oracle_*.py):

* philox4x64_10      -- pinned: equals numpy's Philox bit generator (a
                        published Philox4x64-10 implementation) on the same
                        key and counter.
* pst_sample         -- pinned: radial law P(|p| <= a) = a^6, E[p p^T] = I/8,
                        sign symmetry, acceptance rate pi^3/384, exact
                        2^-24 lattice, row 0 = origin.
* chart_delta / pose_retract / particle_pose
                     -- pinned: closed-form rotations (axis-angle),
                        orthonormality, identity at u = 0, composition with
                        an independent matrix product.
* unproject          -- pinned: noise-free analytic render -> every point
                        lies on the analytic surface.
* overlap            -- pinned: identity motion keeps every point; pure
                        forward translation keeps exactly the analytically
                        predicted set.
* fitness            -- pinned: analytic plane field F(d) = (d/mu)^2
                        (trilinear exact on a linear field); 1-Lipschitz
                        bound at the true pose (nearest); all-outside -> 1;
                        voxel index brute force.  Sums: binary64 mode
                        (Neumaier) vs math.fsum; binary32 mode (the 2^-39
                        grid) equals the exact rational sum of the terms
                        rounded to the grid, is within m 2^-40 of math.fsum
                        and does not change under any permutation of the
                        points.
* exp_rho            -- pinned: within 1 ulp of math.exp over [-745, 0] and
                        exact at 0.
  (kahan=False)         the plain binary32 sum: within the recursive-
                        summation bound (m-1) 2^-24 sum v^2 of math.fsum; a
                        constructed case where it loses exactly the terms
                        below half an ulp of the running sum.
* pst_update         -- pinned: single-member APS reproduces that particle;
                        symmetric APS -> zero step; empty APS and
                        TSDF-not-built corner cases; permutation invariance.
* track_frame        -- pinned: brute-force 6D grid search on a tiny scene
                        within the paper's 20 iterations (both threshold
                        readings); convergence to the true pose on the small
                        frame; an independent replay of the loop through
                        pst_update with the threshold carried as Eq. wafit
                        reads (centre fitness at k = 1, then rho~ of the last
                        non-empty iteration, unchanged across empty ones)
                        equals it bit for bit.
* set_threads        -- fitness over particle ranges and fusion over
                        z-slices on host threads: equal bit for bit to one
                        thread.
* integrate          -- pinned: fronto-parallel plane closed form; fused
                        zero crossing vs analytic surface.
* track_frame levels -- pinned: identical levels reproduce the single
  (multi-resolution)    resolution tracker bit for bit; with the centre
                        threshold a K-iteration schedule equals K chained
                        one-iteration single-resolution runs; the paper's
                        schedule converges on the small frame.
* pst_update flags   -- pinned: the worked example with the isotropic or
  (rescaling ablation)  the anisotropic part of Eq. rsinter switched off.
* pst_poisson        -- pinned: r_min = 0 gives the i.i.d. template bit for
                        bit; exact minimum spacing; every rejected candidate
                        lies within r_min of an earlier accepted point;
                        budget exhaustion; uniform-like moments.
* raycast            -- pinned: analytic render of a scene at the same pose
                        within half a voxel; plane exact; misses are 0.
* proposal_features  -- pinned: closed forms on constant frames (clamped
                        difference, missing samples, velocity, padding).
* pfo_resample / pso_move / swarm_frame (comparison optimisers of the
  Sec. 5 ablation)   -- pinned: a hand-worked resampling example; equal
                        weights give the identity; one dominant weight takes
                        every slot; copy counts within one of n w_i / W; a
                        hand-worked PSO step with the velocity clamp; with no
                        motion (sigma = 0, or c1 = c2 = 0 from rest) the
                        result is the brute-force best of the initial set;
                        the best fitness never decreases; both converge on
                        the small frame.
* mlp (oracle/mlp.py) -- pinned: central differences of the loss; GELU
                        closed forms; the NLL minimiser is the sample mean
                        and log standard deviation; Adam's first step.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rose_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

F64 = 0
F32 = 1
NEAREST = 0
TRILINEAR = 1
NO_OVERLAP = 1
NO_NORMALIZE = 2
CENTRE_THRESHOLD = 4
ISO_ONLY = 8
ANISO_ONLY = 16
NO_KAHAN = 32
SWARM_PFO = 0
SWARM_PSO = 1


def _cpu_has_fma() -> bool:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("flags"):
                    return " fma " in line + " "
    except OSError:
        pass
    return False


def build(force: bool = True) -> str:
    """Compile rose_oracle.c into liboracle.so (gcc, -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread"]
        if _cpu_has_fma():
            cmd.append("-mfma")  # fmaf() inlines to the (correctly rounded) hardware instruction
        cmd += ["-o", tmp, _SRC, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _TrackParams(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("early_stop", C.c_int32), ("stride", C.c_int32),
                ("lookup", C.c_int32), ("flags", C.c_int32), ("prec", C.c_int32),
                ("levels", C.c_int32), ("level_n", C.c_int32 * 4), ("level_stride", C.c_int32 * 4),
                ("beta", C.c_double), ("eps", C.c_double), ("tau", C.c_double), ("stop_tol", C.c_double)]


class _SwarmParams(C.Structure):
    _fields_ = [("method", C.c_int32), ("iters", C.c_int32), ("stride", C.c_int32), ("lookup", C.c_int32),
                ("flags", C.c_int32), ("prec", C.c_int32), ("tau", C.c_double), ("r_init", C.c_double * 6),
                ("sigma", C.c_double * 6), ("w_start", C.c_double), ("w_end", C.c_double), ("c1", C.c_double),
                ("c2", C.c_double), ("vmax", C.c_double * 6)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            lib = C.CDLL(_LIB)
            P = C.c_void_p
            lib.orc_set_threads.argtypes = [C.c_int32]
            lib.orc_get_threads.restype = C.c_int32
            lib.orc_exp.argtypes = [C.c_double]
            lib.orc_exp.restype = C.c_double
            lib.orc_philox4x64_10.argtypes = [P, P, P]
            lib.orc_pst_sample.argtypes = [C.c_int32, C.c_uint64, P]
            lib.orc_pst_sample.restype = C.c_int
            lib.orc_chart_delta.argtypes = [P, P, P]
            lib.orc_pose_retract.argtypes = [P, P, P, P, P]
            lib.orc_particle_pose.argtypes = [P, P, P, P, P]
            lib.orc_unproject.argtypes = [P, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float,
                                          C.c_int32, C.c_int, P]
            lib.orc_unproject.restype = C.c_int
            lib.orc_overlap.argtypes = [P, C.c_int32, P, P, C.c_float, C.c_float, C.c_float, C.c_float,
                                        C.c_int32, C.c_int32, P, C.c_int, P]
            lib.orc_overlap.restype = C.c_int
            lib.orc_fitness.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, C.c_int32, P, P,
                                        C.c_int32, C.c_int32, C.c_int, C.c_int, P]
            lib.orc_fitness_ex.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, C.c_int32, P, P,
                                           C.c_int32, C.c_int32, C.c_int, C.c_int, C.c_int, P]
            lib.orc_voxel_indices.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, C.c_int32, P,
                                              C.c_int32, P]
            lib.orc_pst_poisson.argtypes = [C.c_int32, C.c_uint64, C.c_double, C.c_int32, P, P]
            lib.orc_pst_poisson.restype = C.c_int32
            lib.orc_pst_update.argtypes = [P, P, C.c_int32, P, P, P, C.c_double, C.c_double, C.c_double,
                                           C.c_int32, C.c_double, P, P, P, P, P, C.c_int32]
            lib.orc_pst_update.restype = C.c_int
            lib.orc_track_frame.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, P, C.c_int32,
                                            C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, P, C.c_int32,
                                            P, P, P, P, P, C.c_int32, C.POINTER(_TrackParams), P, P, P, P, P,
                                            P, P, P, P, P, P, P]
            lib.orc_track_frame.restype = C.c_int
            lib.orc_integrate.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, C.c_float,
                                          C.c_float, P, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float,
                                          C.c_float, P, P, C.c_int]
            lib.orc_integrate.restype = C.c_int64
            lib.orc_pfo_resample.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_double, P]
            lib.orc_pso_move.argtypes = [P, P, P, P, P, C.c_int32, C.c_float, C.c_float, C.c_float, P]
            lib.orc_swarm_frame.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, C.c_int32,
                                            C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, P, C.c_int32,
                                            P, P, C.POINTER(_SwarmParams), P, P, P, P, P, P, P, P, P, P]
            lib.orc_swarm_frame.restype = C.c_int
            lib.orc_raycast.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, P, C.c_int32,
                                        C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_double, P]
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------- wrappers
def set_threads(n: int) -> None:
    """Host threads of the oracle's fitness (contiguous particle ranges) and
    fusion (z-slices); results do not depend on it.  Process-wide."""
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


class threads:
    """Context manager: run the enclosed oracle calls on n host threads."""

    def __init__(self, n: int):
        self.n = int(n)

    def __enter__(self):
        self.prev = get_threads()
        set_threads(self.n)
        return self

    def __exit__(self, *exc):
        set_threads(self.prev)
        return False


def host_threads() -> int:
    """Threads this process may run on (its CPU affinity)."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def philox4x64_10(ctr, key) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib.orc_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def exp_rho(x) -> np.ndarray:
    """The oracle's exp (orc_exp: Cody-Waite reduction, degree-13 Taylor
    polynomial by Horner's rule with fma, 2^k scaling), elementwise."""
    lib = _load()
    xs = np.atleast_1d(np.asarray(x, dtype=np.float64))
    return np.array([lib.orc_exp(float(v)) for v in xs.ravel()]).reshape(xs.shape)


def pst_sample(n: int, seed: int):
    """(n, 6) float32 template, and the number of rows that hit the cap."""
    lib = _load()
    out = np.zeros((n, 6), dtype=np.float32)
    capped = lib.orc_pst_sample(int(n), C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), _p(out))
    return out, int(capped)


def chart_delta(u):
    lib = _load()
    u = _f64(u)
    q = np.zeros(4)
    t = np.zeros(3)
    lib.orc_chart_delta(_p(u), _p(q), _p(t))
    return q, t


def pose_retract(qc, tc, u):
    lib = _load()
    qc, tc, u = _f64(qc), _f64(tc), _f64(u)
    q = np.zeros(4)
    t = np.zeros(3)
    lib.orc_pose_retract(_p(qc), _p(tc), _p(u), _p(q), _p(t))
    return q, t


def particle_poses(qc, tc, r, pst) -> np.ndarray:
    """(n, 3, 4) float64 camera->world transforms of the PST particles."""
    lib = _load()
    qc, tc, r = _f64(qc), _f64(tc), _f64(r)
    pst = _f32(pst)
    n = pst.shape[0]
    T = np.zeros((n, 3, 4))
    for i in range(n):
        lib.orc_particle_pose(_p(qc), _p(tc), _p(r), _p(pst[i]), _p(T[i]))
    return T


def unproject(depth, K, stride: int, prec: int = F32) -> np.ndarray:
    lib = _load()
    depth = _f32(depth)
    H, W = depth.shape
    mmax = ((H + stride - 1) // stride) * ((W + stride - 1) // stride)
    out = np.zeros((max(mmax, 1), 3), dtype=np.float32)
    m = lib.orc_unproject(_p(depth), W, H, K.fx, K.fy, K.cx, K.cy, stride, prec, _p(out))
    return out[:m].copy()


def _prev_depth(prev_depth, K):
    if prev_depth is None:
        return None
    d = _f32(prev_depth)
    if d.shape != (K.height, K.width):
        raise ValueError(f"prev_depth must be {K.height} x {K.width}")
    return d


def overlap(pts, Tc, Tprev, K, prec: int = F32, prev_depth=None) -> np.ndarray:
    """Overlap mask (Eq. validness); prev_depth: optional depth of frame
    t-1, whose nearest pixel must then hold a valid depth as well."""
    lib = _load()
    pts = _f32(pts)
    Tc = _f64(np.asarray(Tc)[:3, :4])
    Tprev = _f64(np.asarray(Tprev)[:3, :4])
    mask = np.zeros(max(len(pts), 1), dtype=np.uint8)
    pd = _prev_depth(prev_depth, K)
    lib.orc_overlap(_p(pts), len(pts), _p(Tc), _p(Tprev), K.fx, K.fy, K.cx, K.cy, K.width, K.height,
                    None if pd is None else _p(pd), prec, _p(mask))
    return mask[:len(pts)].astype(bool)


def fitness(psi, vox, origin, pts, T, lookup: int = NEAREST, prec: int = F32, mask=None,
            normalize: bool = True, kahan: bool = True) -> np.ndarray:
    """F_i (float64) for transforms T (n, 3, 4) over points pts (m, 3).

    psi: (nz, ny, nx) float32 normalised TSDF.  kahan=False: the plain
    binary32 sum in point order ("No Kahan" of the Sec. 5 ablation)."""
    lib = _load()
    psi = _f32(psi)
    nz, ny, nx = psi.shape
    pts = _f32(pts).reshape(-1, 3)
    T = _f64(np.asarray(T).reshape(-1, 3, 4))
    org = _f32(origin)
    F = np.zeros(max(len(T), 1))
    mk = None
    if mask is not None:
        mk = np.ascontiguousarray(mask, dtype=np.uint8)
    lib.orc_fitness_ex(_p(psi), nx, ny, nz, float(vox), _p(org), _p(pts), len(pts),
                       _p(mk) if mk is not None else None, _p(T), len(T), lookup, prec, int(normalize),
                       int(not kahan), _p(F))
    return F[:len(T)].copy()


def voxel_indices(dims, vox, origin, pts, T) -> np.ndarray:
    lib = _load()
    nx, ny, nz = dims
    pts = _f32(pts).reshape(-1, 3)
    T = _f64(np.asarray(T).reshape(-1, 3, 4))
    org = _f32(origin)
    idx = np.zeros((len(T), len(pts)), dtype=np.int64)
    lib.orc_voxel_indices(nx, ny, nz, float(vox), _p(org), _p(pts), len(pts), _p(T), len(T), _p(idx))
    return idx


def pst_poisson(n: int, seed: int, r_min: float, max_cand: int):
    """6D Poisson-disk template by dart throwing over the i.i.d. sampler's
    stream; returns (n x 6 float32, rows accepted, candidates drawn)."""
    lib = _load()
    out = np.zeros((n, 6), dtype=np.float32)
    drawn = np.zeros(1, dtype=np.int32)
    got = lib.orc_pst_poisson(int(n), int(seed), float(r_min), int(max_cand), _p(out), _p(drawn))
    return out, int(got), int(drawn[0])


def pst_update(F, pst, r, qc, tc, tau=1.0, beta=0.1, eps=1e-3, tsdf_built=True, rho_thr=None, flags=0):
    lib = _load()
    F = _f64(F)
    pst = _f32(pst)
    r, qc, tc = _f64(r), _f64(qc), _f64(tc)
    r_out, q_out, t_out, us = np.zeros(6), np.zeros(4), np.zeros(3), np.zeros(6)
    rt = np.zeros(1)
    if rho_thr is None:
        rho_thr = float(np.exp(-F[0] / tau))
    aps = lib.orc_pst_update(_p(F), _p(pst), len(F), _p(r), _p(qc), _p(tc), tau, beta, eps, int(tsdf_built),
                             float(rho_thr), _p(r_out), _p(q_out), _p(t_out), _p(rt), _p(us), int(flags))
    return dict(aps=int(aps), r=r_out, q=q_out, t=t_out, rho_tilde=float(rt[0]), u_star=us)


def track_frame(psi, vox, origin, depth, K, pst, q_prev, t_prev, r_init, q_init=None, t_init=None,
                tsdf_built=True, max_iters=20, early_stop=False, stride=4, lookup=NEAREST, flags=0, prec=F32,
                beta=0.1, eps=1e-3, tau=1.0, stop_tol=1e-6, levels=None, prev_depth=None):
    """One frame of Alg. 1.  levels: optional multi-resolution schedule
    [(n_particles, stride), ...] used in turn across the iterations (the
    particles of a level are the first n rows of `pst`).  prev_depth:
    optional depth of frame t-1 for the stricter overlap test (see
    overlap)."""
    lib = _load()
    psi = _f32(psi)
    nz, ny, nx = psi.shape
    depth = _f32(depth)
    H, W = depth.shape
    pst = _f32(pst)
    q_prev, t_prev, r_init = _f64(q_prev), _f64(t_prev), _f64(r_init)
    q_init = q_prev if q_init is None else _f64(q_init)
    t_init = t_prev if t_init is None else _f64(t_init)
    lv = list(levels or [])
    if len(lv) > 4:
        raise ValueError("at most 4 levels")
    ln = (C.c_int32 * 4)(*([int(a) for a, _ in lv] + [0] * (4 - len(lv))))
    ls = (C.c_int32 * 4)(*([int(b) for _, b in lv] + [0] * (4 - len(lv))))
    P = _TrackParams(max_iters, int(early_stop), stride, lookup, flags, prec, len(lv), ln, ls, beta, eps, tau,
                     stop_tol)
    q_out, t_out, r1 = np.zeros(4), np.zeros(3), np.zeros(6)
    rho, iters = np.zeros(1), np.zeros(1, dtype=np.int32)
    aps = np.zeros(32, dtype=np.int32)
    rho_it = np.zeros(32)
    npts, nov = np.zeros(1, dtype=np.int32), np.zeros(1, dtype=np.int32)
    nov_it, rc_it, thr_it = np.zeros(32, dtype=np.int32), np.zeros(32), np.zeros(32)
    org = _f32(origin)
    pd = _prev_depth(prev_depth, K)
    rc = lib.orc_track_frame(_p(psi), nx, ny, nz, float(vox), _p(org), _p(depth),
                             None if pd is None else _p(pd), W, H, K.fx, K.fy, K.cx, K.cy,
                             _p(pst), len(pst), _p(q_prev), _p(t_prev), _p(q_init), _p(t_init), _p(r_init),
                             int(tsdf_built), C.byref(P), _p(q_out), _p(t_out), _p(r1), _p(rho), _p(iters),
                             _p(aps), _p(rho_it), _p(npts), _p(nov), _p(nov_it), _p(rc_it), _p(thr_it))
    it = int(iters[0])
    k = min(it, 32)
    return dict(status=int(rc), q=q_out, t=t_out, r1=r1, rho=float(rho[0]), iters=it,
                aps=aps[:k].copy(), rho_iter=rho_it[:k].copy(), n_points=int(npts[0]),
                n_overlap_last=int(nov[0]), n_overlap=nov_it[:k].copy(), rho_centre=rc_it[:k].copy(),
                thr=thr_it[:k].copy())


def integrate(psi, wgt, vox, origin, mu, depth, K, q, t, w_max=128.0, prec: int = F32) -> int:
    """In-place fusion of one depth frame into (psi, wgt), both (nz, ny, nx)
    float32 C-contiguous arrays.  Returns the number of updated voxels."""
    lib = _load()
    assert psi.dtype == np.float32 and wgt.dtype == np.float32
    assert psi.flags.c_contiguous and wgt.flags.c_contiguous
    nz, ny, nx = psi.shape
    depth = _f32(depth)
    H, W = depth.shape
    q, t = _f64(q), _f64(t)
    org = _f32(origin)
    return int(lib.orc_integrate(_p(psi), _p(wgt), nx, ny, nz, float(vox), _p(org), float(mu), float(w_max),
                                 _p(depth), W, H, K.fx, K.fy, K.cx, K.cy, _p(q), _p(t), prec))


def pose_mat(q, t) -> np.ndarray:
    """4x4 camera->world matrix of (q, t), via the oracle's own quaternion
    formula (binary64)."""
    qd, td = _f64(q), _f64(t)
    T = np.zeros((3, 4))
    lib = _load()
    zero_r = np.zeros(6)
    zero_p = np.zeros(6, dtype=np.float32)
    lib.orc_particle_pose(_p(qd), _p(td), _p(zero_r), _p(zero_p), _p(T))
    M = np.eye(4)
    M[:3, :] = T
    return M


def raycast(psi, vox, origin, q, t, K, near=0.2, far=8.0, step=None) -> np.ndarray:
    """Depth (H, W) float32 of the TSDF rendered at pose (q, t) through the
    intrinsics K (binary32 intrinsics widened to binary64)."""
    lib = _load()
    psi = _f32(psi)
    nz, ny, nx = psi.shape
    q, t = _f64(q), _f64(t)
    org = _f32(origin)
    out = np.zeros((K.height, K.width), np.float32)
    st = float(np.float32(vox)) / 2 if step is None else step
    f32 = lambda v: float(np.float32(v))  # noqa: E731
    lib.orc_raycast(_p(psi), nx, ny, nz, float(vox), _p(org), _p(q), _p(t), K.width, K.height, f32(K.fx), f32(K.fy),
                    f32(K.cx), f32(K.cy), float(near), float(far), float(st), _p(out))
    return out


def proposal_features(depth, render, scale: int, velocity, dim: int) -> np.ndarray:
    """Input vector of the learned proposal: depth residual on the low-res
    grid (the full-res sample at (scale u + scale/2, scale v + scale/2)
    minus the rendered model depth, clamped to +-0.5 m, 0 where either is
    missing), then the 6D previous velocity, then zeros up to dim."""
    depth = np.asarray(depth, np.float32)
    render = np.asarray(render, np.float32)
    h, w = render.shape
    H, W = depth.shape
    out = np.zeros(dim, np.float32)
    for v in range(h):
        for u in range(w):
            U, V = scale * u + scale // 2, scale * v + scale // 2
            d = depth[V, U] if (U < W and V < H) else np.float32(0)
            m = render[v, u]
            if d > 0 and m > 0:
                out[v * w + u] = min(np.float32(0.5), max(np.float32(-0.5), np.float32(d - m)))
    out[h * w:h * w + 6] = np.asarray(velocity, np.float64).astype(np.float32)
    return out


# ------------------------------------------- comparison optimisers (Sec. 5)
def pfo_resample(F, F_best: float, u: float, tau: float = 1.0) -> np.ndarray:
    """Ancestors (int32, n) of systematic resampling with the weights
    exp(-(F_i - F_best)/tau) and offset u in [0, 1)."""
    lib = _load()
    F = _f64(F)
    anc = np.zeros(max(len(F), 1), dtype=np.int32)
    lib.orc_pfo_resample(_p(F), len(F), float(F_best), float(tau), float(u), _p(anc))
    return anc[:len(F)].copy()


def pso_move(x, v, p, g, R, w: float, c1: float, c2: float, vmax):
    """One PSO velocity/position step; returns the new (x, v) (float32)."""
    lib = _load()
    x, v, p = _f32(x).copy(), _f32(v).copy(), _f32(p)
    g, R, vm = _f32(g), _f32(R), _f32(vmax)
    n = x.shape[0]
    lib.orc_pso_move(_p(x), _p(v), _p(p), _p(g), _p(R), n, float(w), float(c1), float(c2), _p(vm))
    return x, v


def swarm_frame(method: int, psi, vox, origin, depth, K, pst, q_prev, t_prev, draws, offsets=None, iters=20,
                stride=4, lookup=NEAREST, flags=0, prec=F32, tau=1.0, r_init=(0.1,) * 6, sigma=None,
                w_start=0.9, w_end=0.4, c1=2.0, c2=2.0, vmax=None):
    """One frame of vanilla PFO (method SWARM_PFO) or PSO (SWARM_PSO) from
    c_0 = (q_prev, t_prev).  draws: PFO (iters, n, 6) standard normals, PSO
    (iters, n, 12) uniforms; offsets: PFO (iters,) uniforms.  sigma defaults
    to r_init / sqrt(8) (the per-axis spread of the initial set), vmax to
    r_init."""
    lib = _load()
    psi = _f32(psi)
    nz, ny, nx = psi.shape
    depth = _f32(depth)
    H, W = depth.shape
    pst = _f32(pst)
    n = len(pst)
    r_init = np.asarray(r_init, np.float64)
    sigma = r_init / np.sqrt(8.0) if sigma is None else np.asarray(sigma, np.float64)
    vmax = r_init if vmax is None else np.asarray(vmax, np.float64)
    d6 = lambda a: (C.c_double * 6)(*[float(e) for e in a])  # noqa: E731
    P = _SwarmParams(method, iters, stride, lookup, flags, prec, tau, d6(r_init), d6(sigma), w_start, w_end, c1,
                     c2, d6(vmax))
    cols = 6 if method == SWARM_PFO else 12
    dr = _f32(draws).reshape(-1)
    assert dr.size >= iters * n * cols, "draws too small"
    off = _f32(np.zeros(iters) if offsets is None else offsets)
    q_out, t_out, rho = np.zeros(4), np.zeros(3), np.zeros(1)
    rb, rm = np.zeros(32), np.zeros(32)
    bi, nov, npts = np.zeros(32, np.int32), np.zeros(32, np.int32), np.zeros(1, np.int32)
    org = _f32(origin)
    q_prev, t_prev = _f64(q_prev), _f64(t_prev)
    rc = lib.orc_swarm_frame(_p(psi), nx, ny, nz, float(vox), _p(org), _p(depth), W, H, K.fx, K.fy, K.cx, K.cy,
                             _p(pst), n, _p(q_prev), _p(t_prev), C.byref(P), _p(dr), _p(off), _p(q_out), _p(t_out),
                             _p(rho), _p(rb), _p(rm), _p(bi), _p(nov), _p(npts))
    k = iters if rc == 0 else 0
    return dict(status=int(rc), q=q_out, t=t_out, rho=float(rho[0]), rho_best=rb[:k].copy(), rho_mean=rm[:k].copy(),
                best_index=bi[:k].copy(), n_overlap=nov[:k].copy(), n_points=int(npts[0]))
