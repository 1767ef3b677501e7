"""Pinhole cameras, poses and depth rendering for the synthetic inputs.

Camera frame: x right, y down, z forward (z-depth in metres).  A pose maps
camera to world: X = R x + t.  Quaternions are (w, x, y, z), Hamilton
convention, stored with w >= 0.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .scene import Scene


@dataclasses.dataclass(frozen=True)
class Intrinsics:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    @staticmethod
    def centred(width: int, height: int, f: float) -> "Intrinsics":
        # integer pixel centres: cx = W/2 - 1/2, cy = H/2 - 1/2
        return Intrinsics(width, height, float(f), float(f), width / 2.0 - 0.5, height / 2.0 - 0.5)


def quat_to_mat(q) -> np.ndarray:
    w, x, y, z = [float(v) for v in q]
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def mat_to_quat(R) -> np.ndarray:
    """Rotation matrix -> unit quaternion (w >= 0), Shepperd's method."""
    R = np.asarray(R, dtype=np.float64)
    tr = np.trace(R)
    cand = [tr, R[0, 0], R[1, 1], R[2, 2]]
    i = int(np.argmax(cand))
    if i == 0:
        s = 2.0 * np.sqrt(1.0 + tr)
        q = [0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s]
    elif i == 1:
        s = 2.0 * np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2])
        q = [(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s]
    elif i == 2:
        s = 2.0 * np.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2])
        q = [(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s]
    else:
        s = 2.0 * np.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1])
        q = [(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s]
    q = np.asarray(q)
    q /= np.linalg.norm(q)
    if q[0] < 0:
        q = -q
    return q


def axis_angle(axis, angle) -> np.ndarray:
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * (K @ K)


def look_rotation(forward, up_hint=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Camera->world rotation whose z axis is `forward` (y axis points down)."""
    f = np.asarray(forward, dtype=np.float64)
    f = f / np.linalg.norm(f)
    up = np.asarray(up_hint, dtype=np.float64)
    if abs(f @ up) > 0.95:
        up = np.array([1.0, 0.0, 0.0]) if abs(f[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    x = np.cross(f, up)  # right = forward x up  (y down)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    return np.stack([x, y, f], axis=1)


@dataclasses.dataclass
class Pose:
    R: np.ndarray  # (3,3) camera->world
    t: np.ndarray  # (3,)

    @property
    def q(self) -> np.ndarray:
        return mat_to_quat(self.R)

    def mat(self) -> np.ndarray:
        T = np.eye(4)
        T[:3, :3] = self.R
        T[:3, 3] = self.t
        return T

    def as_3x4(self) -> np.ndarray:
        return self.mat()[:3, :]

    @staticmethod
    def from_qt(q, t) -> "Pose":
        return Pose(quat_to_mat(q), np.asarray(t, dtype=np.float64))


def pixel_rays(K: Intrinsics) -> np.ndarray:
    """Camera-frame ray directions with unit z: ((u-cx)/fx, (v-cy)/fy, 1),
    row-major (H*W, 3)."""
    u = np.arange(K.width, dtype=np.float64)
    v = np.arange(K.height, dtype=np.float64)
    uu, vv = np.meshgrid(u, v, indexing="xy")
    d = np.stack([(uu - K.cx) / K.fx, (vv - K.cy) / K.fy, np.ones_like(uu)], axis=-1)
    return d.reshape(-1, 3)


def render_depth(scene: Scene, K: Intrinsics, pose: Pose, zmin: float = 0.0, zmax: float = np.inf,
                 noise_seed=None, noise_k: float = 0.0) -> np.ndarray:
    """z-depth image (H, W) float32 of the scene seen from `pose`.

    Rays with unit camera-z have ray parameter equal to z-depth.  Depths
    outside (zmin, zmax) are 0 (invalid).  With noise_k > 0, Gaussian noise
    of standard deviation noise_k * z^2 is added (seeded).
    """
    dc = pixel_rays(K)
    # elementwise in a fixed order (a BLAS product may round differently with
    # its threading, which would make the frames differ between runs)
    R = pose.R
    dw = dc[:, 0:1] * R[:, 0] + dc[:, 1:2] * R[:, 1] + dc[:, 2:3] * R[:, 2]
    z = scene.raycast(pose.t, dw)
    if noise_k > 0:
        rng = np.random.default_rng(noise_seed)
        z = z + rng.standard_normal(z.shape) * noise_k * z * z
    z = np.where(np.isfinite(z) & (z > zmin) & (z < zmax), z, 0.0)
    return z.reshape(K.height, K.width).astype(np.float32)
