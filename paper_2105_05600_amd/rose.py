"""Python binding of librose (include/rose.h): argument marshalling only.

Every step of the pose search and the fusion runs in the HIP kernels of
librose.so; this module converts torch tensors (device memory, streams) and
small host structs to the C ABI and raises on a non-OK status.  There is no
CPU fallback: importing this module fails loudly when the library has not
been built.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import re
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librose.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "rose.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"librose.so is not built ({LIB_PATH}); run __graft_entry__.build() "
                      "or python -m paper_2105_05600_amd.build")

_lib = C.CDLL(LIB_PATH)

OK = 0
E_ARG, E_SHAPE, E_DEVICE, E_STATE, E_UNSUPPORTED = -1, -2, -3, -4, -5
F32, F16, SN16 = 0, 1, 2
NEAREST, TRILINEAR = 0, 1
FLAG_NO_OVERLAP, FLAG_NO_NORMALIZE, FLAG_CENTRE_THRESHOLD, FLAG_ISO_ONLY, FLAG_ANISO_ONLY = 1, 2, 4, 8, 16
FLAG_NO_KAHAN = 32
MAX_ITERS = 32
MAX_LEVELS = 4


class Camera(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class Pose(C.Structure):
    _fields_ = [("q", C.c_double * 4), ("t", C.c_double * 3)]


class TrackParams(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("early_stop", C.c_int32), ("stride", C.c_int32),
                ("lookup", C.c_int32), ("flags", C.c_int32), ("levels", C.c_int32),
                ("beta", C.c_double), ("eps", C.c_double), ("tau", C.c_double), ("stop_tol", C.c_double),
                ("level_n", C.c_int32 * MAX_LEVELS), ("level_stride", C.c_int32 * MAX_LEVELS)]


class TrackState(C.Structure):
    _fields_ = [("pose", Pose), ("r", C.c_double * 6), ("rho", C.c_double), ("tsdf_built", C.c_int32),
                ("frame", C.c_int32)]


class TrackStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("n_points", C.c_int32), ("n_overlap_last", C.c_int32),
                ("status", C.c_int32), ("aps_size", C.c_int32 * MAX_ITERS),
                ("n_overlap", C.c_int32 * MAX_ITERS), ("rho_iter", C.c_double * MAX_ITERS),
                ("n_particles", C.c_int32 * MAX_ITERS), ("rho_centre", C.c_double * MAX_ITERS),
                ("r_iter", (C.c_double * 6) * MAX_ITERS), ("fit_mode", C.c_int32 * MAX_ITERS)]


class LearnedParams(C.Structure):
    _fields_ = [("low_w", C.c_int32), ("low_h", C.c_int32), ("scale", C.c_int32), ("feature_dim", C.c_int32),
                ("kappa", C.c_double), ("r_min", C.c_double), ("r_max", C.c_double), ("delta", C.c_double),
                ("near_m", C.c_double), ("far_m", C.c_double), ("step_m", C.c_double), ("iters", C.c_int32),
                ("reserved", C.c_int32)]


def learned_params(scale=16, low_w=40, low_h=30, feature_dim=1216, kappa=2.0, r_min=1e-3, r_max=1.0, delta=0.01,
                   near=0.2, far=8.0, step=0.005, iters=0) -> "LearnedParams":
    """iters: iterations of the learned run (0: those of the track
    parameters; the plain fallback always uses the track parameters)."""
    return LearnedParams(low_w, low_h, scale, feature_dim, kappa, r_min, r_max, delta, near, far, step, int(iters), 0)


class SwarmParams(C.Structure):
    _fields_ = [("iters", C.c_int32), ("stride", C.c_int32), ("lookup", C.c_int32), ("flags", C.c_int32),
                ("tau", C.c_double), ("r_init", C.c_double * 6), ("sigma", C.c_double * 6),
                ("w_start", C.c_double), ("w_end", C.c_double), ("c1", C.c_double), ("c2", C.c_double),
                ("vmax", C.c_double * 6)]


class SwarmStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("n_points", C.c_int32), ("n_overlap", C.c_int32 * MAX_ITERS),
                ("best_index", C.c_int32 * MAX_ITERS), ("rho_best", C.c_double * MAX_ITERS),
                ("rho_mean", C.c_double * MAX_ITERS)]


def swarm_params(iters=20, stride=4, lookup=NEAREST, flags=0, tau=1.0, r_init=(0.1,) * 6, sigma=None, w_start=0.9,
                 w_end=0.4, c1=2.0, c2=2.0, vmax=None) -> "SwarmParams":
    """Parameters of the comparison optimisers (vanilla PFO, PSO).  sigma
    defaults to r_init / sqrt(8) (the per-axis spread of the initial set),
    vmax to r_init."""
    r = [float(v) for v in r_init]
    sg = [v / math.sqrt(8.0) for v in r] if sigma is None else [float(v) for v in sigma]
    vm = r if vmax is None else [float(v) for v in vmax]
    d6 = lambda v: (C.c_double * 6)(*v)  # noqa: E731
    return SwarmParams(int(iters), int(stride), int(lookup), int(flags), float(tau), d6(r), d6(sg), float(w_start),
                       float(w_end), float(c1), float(c2), d6(vm))


class Profile(C.Structure):
    _fields_ = [("fitness_ms", C.c_double), ("fitness_launches", C.c_int64), ("fitness_evals", C.c_double),
                ("update_ms", C.c_double), ("update_launches", C.c_int64), ("integrate_ms", C.c_double),
                ("integrate_launches", C.c_int64)]


_P = C.c_void_p
_S = C.c_void_p  # hipStream_t
_sigs = {
    "rose_last_error": ([], C.c_char_p),
    "rose_version": ([], C.c_char_p),
    "tsdf_bytes": ([C.c_int32, C.c_int32, C.c_int32, C.c_int, C.c_int32], C.c_size_t),
    "tsdf_create": ([C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_float, _P, C.c_int, C.c_float, _P, _P, _S,
                     C.POINTER(C.c_void_p)], C.c_int),
    "tsdf_destroy": ([_P], C.c_int),
    "tsdf_integrate": ([_P, _P, C.POINTER(Camera), C.POINTER(Pose), _S], C.c_int),
    "tsdf_export": ([_P, _P, _P, _S], C.c_int),
    "tsdf_import": ([_P, _P, _P, _S], C.c_int),
    "pst_sample": ([C.c_int32, C.c_uint64, _P, _S], C.c_int),
    "pst_particle_poses": ([C.POINTER(Pose), _P, _P, C.c_int32, _P, _S], C.c_int),
    "fitness_eval": ([_P, _P, C.c_int32, _P, C.c_int32, C.c_int, _P, _P, _S], C.c_int),
    "fitness_eval_noalloc": ([_P, _P, C.c_int32, _P, C.c_int32, C.c_int, _P, _P, _S], C.c_int),
    "fitness_eval_noalloc_max_points": ([], C.c_int32),
    "fitness_voxel_indices": ([_P, _P, C.c_int32, _P, C.c_int32, _P, _S], C.c_int),
    "depth_unproject": ([_P, C.POINTER(Camera), C.c_int32, C.c_int32, _P, _P, _S], C.c_int),
    "rose_fitness_set_shape": ([C.c_int32, C.c_int32], C.c_int),
    "rose_fitness_set_switch": ([C.c_float, C.c_float], C.c_int),
    "rose_fitness_set_switch_shape": ([C.c_int32, C.c_int32], C.c_int),
    "tsdf_set_fitness_shape": ([_P, C.c_int32, C.c_int32], C.c_int),
    "tsdf_set_fitness_switch": ([_P, C.c_float, C.c_float, C.c_int32, C.c_int32], C.c_int),
    "tsdf_forget_templates": ([_P], C.c_int),
    "tsdf_template_orders": ([_P], C.c_int32),
    "overlap_mask": ([_P, C.c_int32, C.POINTER(Pose), C.POINTER(Pose), C.POINTER(Camera), _P, _P, _S], C.c_int),
    "pso_track_frame": ([_P, _P, _P, C.POINTER(Camera), _P, C.c_int32, C.POINTER(TrackParams), C.POINTER(Pose), _P,
                         C.POINTER(TrackState), C.POINTER(TrackStats), _S], C.c_int),
    "tsdf_raycast": ([_P, C.POINTER(Pose), C.POINTER(Camera), C.c_double, C.c_double, C.c_double, _P, _S],
                     C.c_int),
    "proposal_features": ([_P, C.POINTER(Camera), _P, C.POINTER(Camera), C.c_int32, _P, C.c_int32, _P, _S],
                          C.c_int),
    "rose_mlp_param_count": ([C.c_int32, C.c_int32, C.c_int32], C.c_int64),
    "rose_mlp_create": ([C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_void_p)], C.c_int),
    "rose_mlp_destroy": ([_P], C.c_int),
    "rose_mlp_forward": ([_P, _P, _P, C.c_int32, _P, _S], C.c_int),
    "rose_mlp_loss_grad": ([_P, _P, _P, _P, C.c_int32, _P, _P, _S], C.c_int),
    "rose_mlp_adam": ([C.c_int64, _P, _P, _P, _P, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, _S],
                      C.c_int),
    "rose_gemm_bf16": ([C.c_int32, C.c_int32, C.c_int32, _P, C.c_int64, C.c_int64, _P, C.c_int64, C.c_int64, _P,
                        C.c_int64, _S], C.c_int),
    "pso_batch_create": ([C.c_int32, _P, _P, _P, _P, _P, C.c_int32, C.POINTER(C.c_void_p)], C.c_int),
    "pso_batch_track": ([_P, _P, _P, _P, _P, _P, _S], C.c_int),
    "pso_batch_destroy": ([_P], C.c_int),
    "rose_batch_set_own_launch": ([C.c_int64], C.c_int),
    "pso_batch_track_learned": ([_P, _P, _P, _P, _P, _P, C.POINTER(LearnedParams), _P, _P, C.POINTER(TrackParams),
                                 _P, _P, _P, _S], C.c_int),
    "rose_chart_log": ([C.POINTER(Pose), C.POINTER(Pose), _P], C.c_int),
    "rose_chart_exp": ([C.POINTER(Pose), _P, C.POINTER(Pose)], C.c_int),
    "pso_track_frame_learned": ([_P, _P, C.POINTER(Camera), _P, C.c_int32, _P, C.c_int32, _P, _P, _P, _P,
                                 C.POINTER(TrackParams), C.POINTER(LearnedParams), C.POINTER(TrackState),
                                 C.POINTER(TrackStats), _P, _S], C.c_int),
    "vanilla_pfo_track_frame": ([_P, _P, C.POINTER(Camera), _P, C.c_int32, C.POINTER(SwarmParams), _P, _P,
                                 C.POINTER(TrackState), C.POINTER(SwarmStats), _S], C.c_int),
    "plain_pso_track_frame": ([_P, _P, C.POINTER(Camera), _P, C.c_int32, C.POINTER(SwarmParams), _P,
                               C.POINTER(TrackState), C.POINTER(SwarmStats), _S], C.c_int),
    "rose_profile_enable": ([C.c_int32], C.c_int),
    "rose_profile_reset": ([], C.c_int),
    "rose_profile_read": ([C.POINTER(Profile)], C.c_int),
    "rose_profile_fitness_launches": ([_P, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
    "pst_poisson": ([C.c_int32, C.c_uint64, C.c_double, C.c_int32, _P, _P, _P, _S], C.c_int),
    "rose_gather_peak": ([_P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_uint32, _P, _S], C.c_int),
    "rose_gather_peak_loads_per_lane": ([], C.c_int32),
    "rose_l2_read_peak": ([_P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, _P, _S], C.c_int),
    "tsdf_rescan": ([_P, _S], C.c_int),
}
for _name, (_args, _res) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class RoseError(RuntimeError):
    def __init__(self, fn: str, status: int):
        msg = _lib.rose_last_error().decode(errors="replace")
        super().__init__(f"{fn} returned {status}: {msg}")
        self.status = status


def _check(fn: str, st: int):
    if st != OK:
        raise RoseError(fn, st)


def header_functions() -> list:
    """Names of the functions include/rose.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z0-9_]+\s*\*?\s*([a-z0-9_]+)\s*\(", txt, flags=re.M)))


def version() -> str:
    return _lib.rose_version().decode()


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def camera(K) -> Camera:
    """Camera struct from any object with fx, fy, cx, cy, width, height."""
    return Camera(float(K.fx), float(K.fy), float(K.cx), float(K.cy), int(K.width), int(K.height))


def pose(q: Sequence[float], t: Sequence[float]) -> Pose:
    p = Pose()
    for i in range(4):
        p.q[i] = float(q[i])
    for i in range(3):
        p.t[i] = float(t[i])
    return p


class Tsdf:
    """A TSDF volume in caller-owned device memory (torch tensors)."""

    _dtypes = {F32: (torch.float32, torch.float32), F16: (torch.float16, torch.int16),
               SN16: (torch.int16, torch.int16)}

    def __init__(self, dims, voxel: float, trunc: float, origin, fmt: int = F32, w_max: float = 128.0,
                 device: str = "cuda", stream=None):
        nx, ny, nz = (int(d) for d in dims)
        nb = _lib.tsdf_bytes(nx, ny, nz, fmt, 0)
        if nb == 0:
            raise RoseError("tsdf_bytes", E_SHAPE)
        pd, wd = self._dtypes[fmt]
        n = nx * ny * nz
        self.psi = torch.empty(n, dtype=pd, device=device)
        self.weight = torch.empty(n, dtype=wd, device=device)
        self.dims = (nx, ny, nz)
        self.voxel = float(voxel)
        self.trunc = float(trunc)
        self.origin = tuple(float(o) for o in origin)
        self.fmt = fmt
        org = (C.c_float * 3)(*self.origin)
        h = C.c_void_p()
        _check("tsdf_create", _lib.tsdf_create(nx, ny, nz, self.voxel, self.trunc, org, fmt, float(w_max),
                                               _ptr(self.psi), _ptr(self.weight), _stream(stream), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.tsdf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def integrate(self, depth: torch.Tensor, K, q, t, stream=None):
        _dev(depth, torch.float32, "depth")
        cam = camera(K)
        if depth.numel() != cam.width * cam.height:
            raise ValueError("depth size does not match the camera")
        p = pose(q, t)
        _check("tsdf_integrate", _lib.tsdf_integrate(self.handle, _ptr(depth), C.byref(cam), C.byref(p),
                                                     _stream(stream)))

    def rescan(self, stream=None):
        """Rebuild the handle's all-+1 brick bits after writing psi directly."""
        _check("tsdf_rescan", _lib.tsdf_rescan(self.handle, _stream(stream)))

    def forget_templates(self):
        """Drop the cached particle schedule orders (waits for the device)."""
        _check("tsdf_forget_templates", _lib.tsdf_forget_templates(self.handle))

    def template_orders(self) -> int:
        """Number of PST templates whose schedule order is cached."""
        return int(_lib.tsdf_template_orders(self.handle))

    def set_fitness_shape(self, particles_per_wave: int, points_per_lane: int):
        """This handle's own fitness launch shape ((0, 0): switching mode;
        (-1, -1): back to the process-wide default)."""
        _check("tsdf_set_fitness_shape",
               _lib.tsdf_set_fitness_shape(self.handle, int(particles_per_wave), int(points_per_lane)))

    def set_fitness_switch(self, footprint_voxels: float, reference_depth_m: float = 3.0, wide=(4, 2)):
        """This handle's switching threshold and points-across shape."""
        _check("tsdf_set_fitness_switch",
               _lib.tsdf_set_fitness_switch(self.handle, float(footprint_voxels), float(reference_depth_m),
                                            int(wide[0]), int(wide[1])))

    def export(self, stream=None):
        nx, ny, nz = self.dims
        psi = torch.empty((nz, ny, nx), dtype=torch.float32, device=self.psi.device)
        w = torch.empty((nz, ny, nx), dtype=torch.float32, device=self.psi.device)
        _check("tsdf_export", _lib.tsdf_export(self.handle, _ptr(psi), _ptr(w), _stream(stream)))
        return psi, w

    def load(self, psi_lin: torch.Tensor, w_lin: Optional[torch.Tensor] = None, stream=None):
        _dev(psi_lin, torch.float32, "psi")
        if w_lin is not None:
            _dev(w_lin, torch.float32, "weight")
        if psi_lin.numel() != self.psi.numel():
            raise ValueError("psi size does not match the volume")
        _check("tsdf_import", _lib.tsdf_import(self.handle, _ptr(psi_lin), _ptr(w_lin), _stream(stream)))


def pst_sample(n: int, seed: int, device: str = "cuda", stream=None) -> torch.Tensor:
    out = torch.empty((n, 6), dtype=torch.float32, device=device)
    _check("pst_sample", _lib.pst_sample(int(n), C.c_uint64(int(seed) & (2**64 - 1)), _ptr(out), _stream(stream)))
    return out


def particle_poses(qc, tc, r, pst: torch.Tensor, stream=None) -> torch.Tensor:
    _dev(pst, torch.float32, "pst")
    n = pst.shape[0]
    T = torch.empty((n, 3, 4), dtype=torch.float64, device=pst.device)
    c = pose(qc, tc)
    rr = (C.c_double * 6)(*[float(v) for v in r])
    _check("pst_particle_poses", _lib.pst_particle_poses(C.byref(c), rr, _ptr(pst), n, _ptr(T), _stream(stream)))
    return T


def fitness_eval(vol: Tsdf, pts: torch.Tensor, T: torch.Tensor, lookup: int = NEAREST, stream=None):
    _dev(pts, torch.float32, "pts")
    _dev(T, torch.float32, "T")
    m = pts.shape[0]
    n = T.shape[0]
    F = torch.empty(n, dtype=torch.float32, device=T.device)
    rho = torch.empty(n, dtype=torch.float32, device=T.device)
    _check("fitness_eval", _lib.fitness_eval(vol.handle, _ptr(pts) if m else None, m, _ptr(T), n, lookup, _ptr(F),
                                             _ptr(rho), _stream(stream)))
    return F, rho


def fitness_eval_noalloc(vol: Tsdf, pts: torch.Tensor, T: torch.Tensor, F: torch.Tensor, rho: torch.Tensor,
                         lookup: int = NEAREST, stream=None):
    """fitness_eval into caller-given F and rho (n float32 each) with the
    library's fixed scratch: no device allocation by the library."""
    _dev(pts, torch.float32, "pts")
    _dev(T, torch.float32, "T")
    _dev(F, torch.float32, "F")
    _dev(rho, torch.float32, "rho")
    m = pts.shape[0]
    n = T.shape[0]
    if F.numel() < n or rho.numel() < n:
        raise ValueError("F and rho need n elements")
    _check("fitness_eval_noalloc", _lib.fitness_eval_noalloc(vol.handle, _ptr(pts) if m else None, m, _ptr(T), n,
                                                             lookup, _ptr(F), _ptr(rho), _stream(stream)))


def voxel_indices(vol: Tsdf, pts: torch.Tensor, T: torch.Tensor, stream=None) -> torch.Tensor:
    _dev(pts, torch.float32, "pts")
    _dev(T, torch.float32, "T")
    idx = torch.empty((T.shape[0], pts.shape[0]), dtype=torch.int64, device=T.device)
    _check("fitness_voxel_indices", _lib.fitness_voxel_indices(vol.handle, _ptr(pts), pts.shape[0], _ptr(T),
                                                               T.shape[0], _ptr(idx), _stream(stream)))
    return idx


def depth_unproject(depth: torch.Tensor, K, stride: int, tiled: bool = False, stream=None) -> torch.Tensor:
    _dev(depth, torch.float32, "depth")
    cam = camera(K)
    su = (cam.width + stride - 1) // stride
    sv = (cam.height + stride - 1) // stride
    pts = torch.empty((max(su * sv, 1), 3), dtype=torch.float32, device=depth.device)
    cnt = torch.zeros(1, dtype=torch.int32, device=depth.device)
    _check("depth_unproject", _lib.depth_unproject(_ptr(depth), C.byref(cam), int(stride), int(bool(tiled)), _ptr(pts),
                                                   _ptr(cnt), _stream(stream)))
    return pts[: int(cnt.item())]


def _prev_depth(prev_depth: Optional[torch.Tensor], cam):
    """Device pointer of an optional previous depth frame (NULL when None)."""
    if prev_depth is None:
        return None
    _dev(prev_depth, torch.float32, "prev_depth")
    if prev_depth.numel() != cam.width * cam.height:
        raise ValueError("prev_depth size does not match the camera")
    return _ptr(prev_depth)


def overlap_mask(pts: torch.Tensor, centre, prev, K, stream=None, prev_depth=None) -> torch.Tensor:
    """Overlap mask (Eq. validness); prev_depth: optional depth of frame t-1
    whose nearest pixel must then hold a valid depth as well."""
    _dev(pts, torch.float32, "pts")
    cam = camera(K)
    m = pts.shape[0]
    mask = torch.zeros(max(m, 1), dtype=torch.uint8, device=pts.device)
    c = pose(*centre)
    p = pose(*prev)
    _check("overlap_mask", _lib.overlap_mask(_ptr(pts), m, C.byref(c), C.byref(p), C.byref(cam),
                                             _prev_depth(prev_depth, cam), _ptr(mask), _stream(stream)))
    return mask[:m].bool()


def raycast(vol: Tsdf, q, t, K, near: float = 0.2, far: float = 8.0, step: Optional[float] = None,
            stream=None) -> torch.Tensor:
    cam = camera(K)
    out = torch.empty((cam.height, cam.width), dtype=torch.float32, device=vol.psi.device)
    p = pose(q, t)
    st = vol.voxel / 2 if step is None else step
    _check("tsdf_raycast", _lib.tsdf_raycast(vol.handle, C.byref(p), C.byref(cam), float(near), float(far), float(st),
                                             _ptr(out), _stream(stream)))
    return out


def proposal_features(depth: torch.Tensor, K, render: torch.Tensor, K_low, scale: int, velocity, dim: int,
                      stream=None) -> torch.Tensor:
    _dev(depth, torch.float32, "depth")
    _dev(render, torch.float32, "render")
    cam, cl = camera(K), camera(K_low)
    out = torch.empty(dim, dtype=torch.float32, device=depth.device)
    vel = (C.c_double * 6)(*[float(v) for v in velocity])
    _check("proposal_features", _lib.proposal_features(_ptr(depth), C.byref(cam), _ptr(render), C.byref(cl),
                                                       int(scale), vel, int(dim), _ptr(out), _stream(stream)))
    return out


def track_params(max_iters=20, early_stop=False, stride=4, lookup=NEAREST, flags=0, beta=0.1, eps=1e-3, tau=1.0,
                 stop_tol=1e-6, levels=None) -> TrackParams:
    """levels: optional multi-resolution schedule [(n_particles, stride), ...]
    (2..MAX_LEVELS entries) used in turn across the iterations."""
    lv = list(levels or [])
    if len(lv) > MAX_LEVELS:
        raise ValueError(f"at most {MAX_LEVELS} levels")
    ln = (C.c_int32 * MAX_LEVELS)(*([int(a) for a, _ in lv] + [0] * (MAX_LEVELS - len(lv))))
    ls = (C.c_int32 * MAX_LEVELS)(*([int(b) for _, b in lv] + [0] * (MAX_LEVELS - len(lv))))
    return TrackParams(int(max_iters), int(bool(early_stop)), int(stride), int(lookup), int(flags), len(lv),
                       float(beta), float(eps), float(tau), float(stop_tol), ln, ls)


def track_state(q, t, r, tsdf_built=True, frame=0) -> TrackState:
    st = TrackState()
    st.pose = pose(q, t)
    for i in range(6):
        st.r[i] = float(r[i])
    st.rho = 0.0
    st.tsdf_built = int(bool(tsdf_built))
    st.frame = int(frame)
    return st


def track_frame(vol: Tsdf, depth: torch.Tensor, K, pst: torch.Tensor, params: TrackParams, state: TrackState,
                init_centre=None, init_r=None, stream=None, prev_depth=None) -> dict:
    """Run pso_track_frame; updates `state` in place and returns the stats.
    prev_depth: optional previous depth frame for the stricter overlap test."""
    _dev(depth, torch.float32, "depth")
    _dev(pst, torch.float32, "pst")
    cam = camera(K)
    if depth.numel() != cam.width * cam.height:
        raise ValueError("depth size does not match the camera")
    stats = TrackStats()
    c0 = C.byref(pose(*init_centre)) if init_centre is not None else None
    r0 = (C.c_double * 6)(*[float(v) for v in init_r]) if init_r is not None else None
    st = _lib.pso_track_frame(vol.handle, _ptr(depth), _prev_depth(prev_depth, cam), C.byref(cam), _ptr(pst),
                              pst.shape[0], C.byref(params), c0, r0, C.byref(state), C.byref(stats),
                              _stream(stream))
    _check("pso_track_frame", st)
    it = stats.iters
    return dict(iters=it, n_points=stats.n_points, n_overlap_last=stats.n_overlap_last,
                aps=list(stats.aps_size[:it]), n_overlap=list(stats.n_overlap[:it]),
                rho_iter=list(stats.rho_iter[:it]), n_particles=list(stats.n_particles[:it]),
                rho_centre=list(stats.rho_centre[:it]), r_iter=[list(stats.r_iter[k]) for k in range(it)],
                fit_mode=list(stats.fit_mode[:it]),
                q=list(state.pose.q), t=list(state.pose.t), r1=list(state.r), rho=state.rho)


PFO = 0
PSO = 1


def swarm_track_frame(method: int, vol: Tsdf, depth: torch.Tensor, K, pst: torch.Tensor, params: SwarmParams,
                      state: TrackState, draws: Optional[torch.Tensor], offsets: Optional[torch.Tensor] = None,
                      stream=None) -> dict:
    """One frame of vanilla PFO (method PFO: draws = iters x n x 6 standard
    normals, offsets = iters uniforms) or PSO (method PSO: draws = iters x n
    x 12 uniforms), float32 device tensors; updates `state` in place."""
    _dev(depth, torch.float32, "depth")
    _dev(pst, torch.float32, "pst")
    n = pst.shape[0]
    cols = 6 if method == PFO else 12
    if draws is not None:
        _dev(draws, torch.float32, "draws")
        if draws.numel() < params.iters * n * cols:
            raise ValueError(f"draws must hold iters x n x {cols} values")
    if method == PFO and offsets is not None:
        _dev(offsets, torch.float32, "offsets")
        if offsets.numel() < params.iters:
            raise ValueError("offsets must hold iters values")
    cam = camera(K)
    if depth.numel() != cam.width * cam.height:
        raise ValueError("depth size does not match the camera")
    stats = SwarmStats()
    if method == PFO:
        name = "vanilla_pfo_track_frame"
        st = _lib.vanilla_pfo_track_frame(vol.handle, _ptr(depth), C.byref(cam), _ptr(pst), n, C.byref(params),
                                          _ptr(draws), _ptr(offsets), C.byref(state), C.byref(stats),
                                          _stream(stream))
    elif method == PSO:
        name = "plain_pso_track_frame"
        st = _lib.plain_pso_track_frame(vol.handle, _ptr(depth), C.byref(cam), _ptr(pst), n, C.byref(params),
                                        _ptr(draws), C.byref(state), C.byref(stats), _stream(stream))
    else:
        raise ValueError(f"unknown method {method}")
    _check(name, st)
    it = stats.iters
    return dict(iters=it, n_points=stats.n_points, n_overlap=list(stats.n_overlap[:it]),
                best_index=list(stats.best_index[:it]), rho_best=list(stats.rho_best[:it]),
                rho_mean=list(stats.rho_mean[:it]), q=list(state.pose.q), t=list(state.pose.t), rho=state.rho)


def profile_enable(on: bool = True):
    _check("rose_profile_enable", _lib.rose_profile_enable(int(bool(on))))


def profile_reset():
    _check("rose_profile_reset", _lib.rose_profile_reset())


def pst_poisson(n: int, seed: int, r_min: float, max_candidates: int, stream=None):
    """6D Poisson-disk template (pst_poisson): (n x 6 float32 tensor, rows
    accepted, candidates drawn).  Synchronises the stream to read the
    counts."""
    work = torch.empty((max_candidates + 1) * 6, dtype=torch.float32, device="cuda")
    out = torch.empty((n, 6), dtype=torch.float32, device="cuda")
    res = torch.zeros(2, dtype=torch.int32, device="cuda")
    _check("pst_poisson", _lib.pst_poisson(int(n), int(seed), float(r_min), int(max_candidates), _ptr(work),
                                           _ptr(out), _ptr(res), _stream(stream)))
    got, drawn = res.cpu().tolist()
    return out, int(got), int(drawn)


def poisson_radius(n: int, packing: float = 0.03) -> float:
    """Minimum distance for an n-point template at a given packing fraction
    n (r/2)^6 of the unit ball (0.03: dart throwing draws about 2.3 n to
    2.7 n candidates for n = 1024 to 10240)."""
    return 2.0 * (packing / n) ** (1.0 / 6.0)


def gather_peak(buf: torch.Tensor, region_lines: int, blocks: int, iters: int, sink: torch.Tensor, seed: int = 1,
                stream=None) -> int:
    """Enqueue the gather-rate probe (rose_gather_peak) on `stream`; returns
    the number of 4-byte loads it issues."""
    _dev(buf, torch.float32, "buf")
    _dev(sink, torch.float32, "sink")
    if sink.numel() < blocks:
        raise ValueError("sink needs one float per workgroup")
    _check("rose_gather_peak", _lib.rose_gather_peak(_ptr(buf), buf.numel(), int(region_lines), int(blocks),
                                                     int(iters), int(seed) & 0xFFFFFFFF, _ptr(sink),
                                                     _stream(stream)))
    return int(blocks) * 256 * int(iters) * int(_lib.rose_gather_peak_loads_per_lane())


def l2_read_peak(buf: torch.Tensor, region_f4: int, blocks: int, sweeps: int, sink: torch.Tensor,
                 stream=None) -> int:
    """Enqueue the L2 -> CU read bandwidth probe (rose_l2_read_peak) on
    `stream`; returns the number of bytes it reads."""
    _dev(buf, torch.float32, "buf")
    _dev(sink, torch.float32, "sink")
    if sink.numel() < blocks:
        raise ValueError("sink needs one float per workgroup")
    _check("rose_l2_read_peak", _lib.rose_l2_read_peak(_ptr(buf), buf.numel(), int(region_f4), int(blocks),
                                                       int(sweeps), _ptr(sink), _stream(stream)))
    return int(blocks) * int(sweeps) * int(region_f4) * 16


def profile_fitness_launches() -> np.ndarray:
    """Durations (ms) of the fitness launches timed since the last reset."""
    cnt = C.c_int64(0)
    _check("rose_profile_fitness_launches", _lib.rose_profile_fitness_launches(None, 0, C.byref(cnt)))
    out = np.zeros(max(cnt.value, 1), np.float32)
    _check("rose_profile_fitness_launches",
           _lib.rose_profile_fitness_launches(out.ctypes.data_as(C.c_void_p), cnt.value, C.byref(cnt)))
    return out[: cnt.value].copy()


def profile_read() -> dict:
    p = Profile()
    _check("rose_profile_read", _lib.rose_profile_read(C.byref(p)))
    return {f: getattr(p, f) for f, _ in Profile._fields_}


def gemm_bf16(A: torch.Tensor, B: torch.Tensor, stream=None) -> torch.Tensor:
    """C = A @ B on the matrix cores (BF16 operands, FP32 accumulation).
    A, B: 2-D float32 device tensors with any strides."""
    _dev_any(A, "A")
    _dev_any(B, "B")
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    Cm = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check("rose_gemm_bf16", _lib.rose_gemm_bf16(M, N, K, _ptr(A), A.stride(0), A.stride(1), _ptr(B), B.stride(0),
                                                 B.stride(1), _ptr(Cm), N, _stream(stream)))
    return Cm


def _dev_any(t: torch.Tensor, name: str):
    if not t.is_cuda or t.dtype != torch.float32:
        raise ValueError(f"{name} must be a float32 device tensor")


class Mlp:
    """Activation scratch for the proposal network; parameters, gradients and
    Adam moments are caller-owned flat float32 tensors."""

    def __init__(self, in_dim: int = 1216, hidden: int = 256, out_dim: int = 12, max_batch: int = 1024):
        self.in_dim, self.hidden, self.out_dim, self.max_batch = in_dim, hidden, out_dim, max_batch
        self.n_params = int(_lib.rose_mlp_param_count(in_dim, hidden, out_dim))
        if self.n_params <= 0:
            raise RoseError("rose_mlp_param_count", E_SHAPE)
        h = C.c_void_p()
        _check("rose_mlp_create", _lib.rose_mlp_create(in_dim, hidden, out_dim, max_batch, C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.rose_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, params: dict, device="cuda") -> torch.Tensor:
        """Flatten {W1, b1, W2, b2, W3, b3} (numpy or torch) into the layout."""
        parts = [torch.as_tensor(params[k], dtype=torch.float32).reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
        flat = torch.cat(parts).to(device)
        if flat.numel() != self.n_params:
            raise ValueError("parameter sizes do not match the network")
        return flat.contiguous()

    def unpack(self, flat: torch.Tensor) -> dict:
        i, h, o = self.in_dim, self.hidden, self.out_dim
        shapes = {"W1": (i, h), "b1": (h,), "W2": (h, h), "b2": (h,), "W3": (h, o), "b3": (o,)}
        out, k = {}, 0
        for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
            n = int(np.prod(shapes[name]))
            out[name] = flat[k:k + n].reshape(shapes[name])
            k += n
        return out

    def forward(self, params: torch.Tensor, X: torch.Tensor, stream=None) -> torch.Tensor:
        _dev(params, torch.float32, "params")
        _dev(X, torch.float32, "X")
        B = X.shape[0]
        out = torch.empty((B, self.out_dim), dtype=torch.float32, device=X.device)
        _check("rose_mlp_forward", _lib.rose_mlp_forward(self.handle, _ptr(params), _ptr(X), B, _ptr(out),
                                                         _stream(stream)))
        return out

    def loss_grad(self, params: torch.Tensor, X: torch.Tensor, Y: torch.Tensor, grads: torch.Tensor,
                  loss: torch.Tensor, stream=None):
        for t, n in ((params, "params"), (X, "X"), (Y, "Y"), (grads, "grads"), (loss, "loss")):
            _dev(t, torch.float32, n)
        _check("rose_mlp_loss_grad", _lib.rose_mlp_loss_grad(self.handle, _ptr(params), _ptr(X), _ptr(Y), X.shape[0],
                                                             _ptr(grads), _ptr(loss), _stream(stream)))

    @staticmethod
    def adam(params, grads, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check("rose_mlp_adam", _lib.rose_mlp_adam(params.numel(), _ptr(params), _ptr(grads), _ptr(m), _ptr(v),
                                                   int(step), float(lr), float(beta1), float(beta2), float(eps),
                                                   _stream(stream)))


def set_fitness_shape(particles_per_wave: int, points_per_lane: int):
    _check("rose_fitness_set_shape", _lib.rose_fitness_set_shape(int(particles_per_wave), int(points_per_lane)))


def set_fitness_switch(footprint_voxels: float, reference_depth_m: float = 3.0):
    """Threshold of the switching launch mode (set_fitness_shape(0, 0));
    footprint_voxels = 0 restores the defaults."""
    _check("rose_fitness_set_switch", _lib.rose_fitness_set_switch(float(footprint_voxels), float(reference_depth_m)))


BATCH_OWN_LAUNCH_DEFAULT = 1 << 23


def set_batch_own_launch(min_evals: int):
    """Batches created afterwards give a switching-mode sequence launches of
    its own when n_particles x points per iteration >= min_evals (0: all)."""
    _check("rose_batch_set_own_launch", _lib.rose_batch_set_own_launch(int(min_evals)))


def set_fitness_switch_shape(particles_per_wave: int, points_per_lane: int):
    """Points-across shape of the switching mode (process-wide default)."""
    _check("rose_fitness_set_switch_shape",
           _lib.rose_fitness_set_switch_shape(int(particles_per_wave), int(points_per_lane)))


class Batch:
    """Many sequences tracked in lockstep (pso_batch_*)."""

    def __init__(self, vols, cams, psts, params, use_graph: bool = True):
        self.count = len(vols)
        if not (len(cams) == len(psts) == len(params) == self.count):
            raise ValueError("one camera, template and parameter set per volume")
        self._vols = list(vols)
        self._psts = list(psts)
        H = (C.c_void_p * self.count)(*[v.handle.value for v in vols])
        CA = (Camera * self.count)(*[camera(k) for k in cams])
        PS = (C.c_void_p * self.count)(*[p.data_ptr() for p in psts])
        N = (C.c_int32 * self.count)(*[p.shape[0] for p in psts])
        PR = (TrackParams * self.count)(*params)
        h = C.c_void_p()
        _check("pso_batch_create", _lib.pso_batch_create(self.count, H, CA, PS, N, PR, int(bool(use_graph)),
                                                         C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.pso_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def track(self, depths, states, init_centres=None, init_rs=None, stream=None):
        """states: a ctypes array of TrackState (updated in place); returns
        per-sequence stats dicts."""
        if len(depths) != self.count:
            raise ValueError("one depth frame per sequence")
        D = (C.c_void_p * self.count)(*[d.data_ptr() for d in depths])
        ST = (TrackStats * self.count)()
        IC = None
        if init_centres is not None:
            IC = (Pose * self.count)(*[pose(*c) for c in init_centres])
        IR = None
        if init_rs is not None:
            IR = (C.c_double * (6 * self.count))(*[float(v) for r in init_rs for v in r])
        _check("pso_batch_track", _lib.pso_batch_track(self.handle, D, IC, IR, states, ST, _stream(stream)))
        out = []
        for i in range(self.count):
            s = ST[i]
            it = s.iters
            out.append(dict(status=s.status, iters=it, n_points=s.n_points, aps=list(s.aps_size[:it]),
                            n_overlap=list(s.n_overlap[:it]), fit_mode=list(s.fit_mode[:it]),
                            q=list(states[i].pose.q), t=list(states[i].pose.t), r1=list(states[i].r),
                            rho=states[i].rho))
        return out


def batch_track_learned(batch: "Batch", depths, mlp: "Mlp", mlp_params: torch.Tensor, work: torch.Tensor,
                        velocities, lparams: "LearnedParams", plain_psts, plain_params, states, stream=None):
    """One batched learned frame step (pso_batch_track_learned): the batch's
    own templates and parameters drive the learned runs, plain_psts /
    plain_params the fallbacks.  work: count x (low_w*low_h + feature_dim +
    12) floats.  Returns per-sequence stats dicts with a `fallback` flag."""
    n = batch.count
    if not (len(depths) == len(velocities) == len(plain_psts) == len(plain_params) == n):
        raise ValueError("one depth, velocity, plain template and parameter set per sequence")
    _dev(work, torch.float32, "work")
    need = n * (lparams.low_w * lparams.low_h + lparams.feature_dim + 12)
    if work.numel() < need:
        raise ValueError(f"work needs {need} floats")
    D = (C.c_void_p * n)(*[d.data_ptr() for d in depths])
    V = (C.c_double * (6 * n))(*[float(x) for v in velocities for x in v])
    PP = (C.c_void_p * n)(*[p.data_ptr() for p in plain_psts])
    NP = (C.c_int32 * n)(*[p.shape[0] for p in plain_psts])
    PR = (TrackParams * n)(*plain_params)
    ST = (TrackStats * n)()
    FB = (C.c_int32 * n)()
    _check("pso_batch_track_learned", _lib.pso_batch_track_learned(
        batch.handle, D, mlp.handle, _ptr(mlp_params), _ptr(work), V, C.byref(lparams), PP, NP, PR, states, ST, FB,
        _stream(stream)))
    out = []
    for i in range(n):
        s_ = ST[i]
        it = s_.iters
        out.append(dict(status=s_.status, iters=it, n_points=s_.n_points, aps=list(s_.aps_size[:it]),
                        n_overlap=list(s_.n_overlap[:it]), n_particles=list(s_.n_particles[:it]),
                        q=list(states[i].pose.q), t=list(states[i].pose.t), r1=list(states[i].r),
                        rho=states[i].rho, fallback=bool(FB[i])))
    return out


def chart_log(qa, ta, qb, tb):
    """u with pose_b = pose_a * Delta(u) (the chart of Sec. 3.3)."""
    u = (C.c_double * 6)()
    _check("rose_chart_log", _lib.rose_chart_log(C.byref(pose(qa, ta)), C.byref(pose(qb, tb)), u))
    return list(u)


def chart_exp(qa, ta, u):
    out = Pose()
    uu = (C.c_double * 6)(*[float(v) for v in u])
    _check("rose_chart_exp", _lib.rose_chart_exp(C.byref(pose(qa, ta)), uu, C.byref(out)))
    return list(out.q), list(out.t)


def track_frame_learned(vol: Tsdf, depth: torch.Tensor, K, pst_small: torch.Tensor, pst_plain: torch.Tensor,
                        mlp: "Mlp", mlp_params: torch.Tensor, work: torch.Tensor, velocity, params: TrackParams,
                        lparams: "LearnedParams", state: TrackState, stream=None) -> dict:
    _dev(depth, torch.float32, "depth")
    cam = camera(K)
    stats = TrackStats()
    fb = C.c_int32(0)
    vel = (C.c_double * 6)(*[float(v) for v in velocity])
    _check("pso_track_frame_learned", _lib.pso_track_frame_learned(
        vol.handle, _ptr(depth), C.byref(cam), _ptr(pst_small), pst_small.shape[0], _ptr(pst_plain),
        pst_plain.shape[0], mlp.handle, _ptr(mlp_params), _ptr(work), vel, C.byref(params), C.byref(lparams),
        C.byref(state), C.byref(stats), C.byref(fb), _stream(stream)))
    it = stats.iters
    return dict(iters=it, n_points=stats.n_points, aps=list(stats.aps_size[:it]),
                n_overlap=list(stats.n_overlap[:it]), n_particles=list(stats.n_particles[:it]),
                q=list(state.pose.q), t=list(state.pose.t), r1=list(state.r), rho=state.rho,
                fallback=bool(fb.value))
