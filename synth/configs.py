"""Seeded synthetic workloads.

These stand in for the paper's datasets (ICL-NUIM, TUM RGB-D, ETH3D and
FastCaMo, Sec. 5.1), none of which is used.  The fast-motion sequences
follow the speed ranges the paper reports for its synthetic fast-motion set
(1-4 m/s, about 1-2 rad/s; Tab. speed-info).

* small_frame():  one-frame workload -- 64^3 TSDF at 2 cm (truncation 6 cm)
  of a unit box room with 3 spheres, fused from 5 noise-free 160x120 frames
  (f = 140) looking towards room corners (15 degree jitter); the tracked
  frame is offset from the last fused view by 5 cm and 3 degrees.
* room_sequence(): a 300-frame 640x480 (f = 525) sequence at 30 fps,
  3 m/s and 2 rad/s, through a procedural room of boxes, cylinders and
  spheres, depth noise sigma = 0.002 z^2, for a 512^3 TSDF at 1 cm with a
  15 cm truncation band.
"""
from __future__ import annotations

import dataclasses
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Optional

import numpy as np

from .camera import Intrinsics, Pose, axis_angle, look_rotation, render_depth
from .scene import Scene, procedural_room, unit_box_room


def _random_unit(rng) -> np.ndarray:
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def _cone_direction(rng, base, max_angle) -> np.ndarray:
    base = np.asarray(base, dtype=np.float64)
    perp = np.cross(base, _random_unit(rng))
    perp /= np.linalg.norm(perp)
    ang = rng.uniform(0.0, max_angle)
    return axis_angle(perp, ang) @ base


@dataclasses.dataclass
class SmallFrame:
    scene: Scene
    K: Intrinsics
    dims: tuple
    vox: float
    origin: np.ndarray
    mu: float
    fuse_poses: List[Pose]
    fuse_depths: List[np.ndarray]
    gt_pose: Pose
    depth: np.ndarray  # the tracked frame
    stride: int = 3
    n_particles: int = 1024
    iters: int = 10
    pst_seed: int = 5600


def small_frame(scene_seed: int = 2105, motion_seed: int = 1, offset_m: float = 0.05,
                offset_deg: float = 3.0) -> SmallFrame:
    scene = unit_box_room(scene_seed)
    K = Intrinsics.centred(160, 120, 140.0)
    rng = np.random.default_rng(scene_seed + 1)
    # views towards room corners, so that every frame sees three walls
    bases = [(-1, 1, 1), (1, -1, 1), (-1, -1, -1), (1, 1, -1), (1, 1, 1)]
    poses = []
    for b in bases:
        f = _cone_direction(rng, np.asarray(b, float) / np.sqrt(3.0), np.deg2rad(15.0))
        t = _random_unit(rng) * rng.uniform(0.0, 0.03)
        poses.append(Pose(look_rotation(f), t))
    depths = [render_depth(scene, K, p) for p in poses]
    mrng = np.random.default_rng(motion_seed)
    dirn = _random_unit(mrng)
    axis = _random_unit(mrng)
    last = poses[-1]
    gt = Pose(axis_angle(axis, np.deg2rad(offset_deg)) @ last.R, last.t + offset_m * dirn)
    depth = render_depth(scene, K, gt)
    return SmallFrame(scene, K, (64, 64, 64), 0.02, np.full(3, -0.64), 0.06, poses, depths, gt, depth)


# --------------------------------------------------------------- sequences
def _catmull_rom_closed(P: np.ndarray, samples_per_seg: int) -> np.ndarray:
    n = len(P)
    out = []
    for i in range(n):
        p0, p1, p2, p3 = P[(i - 1) % n], P[i], P[(i + 1) % n], P[(i + 2) % n]
        s = np.linspace(0.0, 1.0, samples_per_seg, endpoint=False)[:, None]
        out.append(0.5 * ((2 * p1) + (-p0 + p2) * s + (2 * p0 - 5 * p1 + 4 * p2 - p3) * s * s
                          + (-p0 + 3 * p1 - 3 * p2 + p3) * s * s * s))
    return np.concatenate(out, axis=0)


@dataclasses.dataclass
class Sequence:
    scene: Scene
    K: Intrinsics
    dims: tuple
    vox: float
    origin: np.ndarray
    mu: float
    poses: List[Pose]
    noise_seed: int
    noise_k: float
    zmin: float
    zmax: float
    stride: int
    n_particles: int
    iters: int
    _cache: Dict[int, np.ndarray] = dataclasses.field(default_factory=dict)

    def __len__(self):
        return len(self.poses)

    def depth(self, i: int) -> np.ndarray:
        if i not in self._cache:
            self._cache[i] = render_depth(self.scene, self.K, self.poses[i], self.zmin, self.zmax,
                                          noise_seed=(self.noise_seed, i), noise_k=self.noise_k)
        return self._cache[i]

    def depths(self, idx, workers: int = 8) -> List[np.ndarray]:
        idx = list(idx)
        todo = [i for i in idx if i not in self._cache]
        if todo:
            with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
                for i, d in zip(todo, ex.map(lambda j: render_depth(
                        self.scene, self.K, self.poses[j], self.zmin, self.zmax,
                        noise_seed=(self.noise_seed, j), noise_k=self.noise_k), todo)):
                    self._cache[i] = d
        return [self._cache[i] for i in idx]


def fast_trajectory(scene: Scene, seed: int, n_frames: int, fps: float, speed: float, ang_speed: float,
                    clearance: float = 0.4) -> List[Pose]:
    """Closed Catmull-Rom path through free-space waypoints (clearance >=
    `clearance`), re-parametrised to constant `speed`; orientation integrates
    a smooth random body angular velocity of constant magnitude `ang_speed`,
    with a weak pull towards the room centre so the view stays inside."""
    rng = np.random.default_rng(seed)
    lo, hi = scene.room_lo, scene.room_hi
    centre = 0.5 * (lo + hi)
    for _attempt in range(200):
        pts = []
        while len(pts) < 8:
            p = rng.uniform(lo + clearance, hi - clearance)
            if scene.sdf(p[None])[0] >= clearance:
                pts.append(p)
        P = np.array(pts)
        ang = np.arctan2(P[:, 1] - centre[1], P[:, 0] - centre[0])
        P = P[np.argsort(ang)]
        curve = _catmull_rom_closed(P, 400)
        if scene.sdf(curve).min() >= 0.6 * clearance:
            break
    else:
        raise RuntimeError("no collision-free path found")
    seg = np.linalg.norm(np.diff(np.concatenate([curve, curve[:1]]), axis=0), axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    L = cum[-1]
    closed = np.concatenate([curve, curve[:1]])
    dt = 1.0 / fps
    # smooth random angular velocity: 3 sinusoids per axis
    freqs = rng.uniform(0.05, 0.4, size=(3, 3))
    phases = rng.uniform(0, 2 * np.pi, size=(3, 3))
    amps = rng.uniform(0.5, 1.0, size=(3, 3))
    t0 = closed[0]
    R = look_rotation(centre - t0)
    poses = []
    for k in range(n_frames):
        s = (speed * k * dt) % L
        i = int(np.searchsorted(cum, s, side="right") - 1)
        i = min(max(i, 0), len(seg) - 1)
        a = (s - cum[i]) / max(seg[i], 1e-12)
        t = closed[i] * (1 - a) + closed[i + 1] * a
        poses.append(Pose(R.copy(), t))
        tk = k * dt
        w = np.array([np.sum(amps[d] * np.sin(2 * np.pi * freqs[d] * tk + phases[d])) for d in range(3)])
        w = w / max(np.linalg.norm(w), 1e-9)
        to_c = centre - t
        to_c = R.T @ (to_c / np.linalg.norm(to_c))  # in camera frame
        pull = np.cross(np.array([0.0, 0.0, 1.0]), to_c)
        w = w + 1.5 * pull
        w = ang_speed * w / max(np.linalg.norm(w), 1e-9)
        ang_k = np.linalg.norm(w) * dt
        R = R @ axis_angle(w, ang_k)
        # re-orthonormalise
        U, _, Vt = np.linalg.svd(R)
        R = U @ Vt
    return poses


def room_sequence(scene_seed: int = 7, traj_seed: int = 11, noise_seed: int = 13, n_frames: int = 300,
                  fps: float = 30.0, speed: float = 3.0, ang_speed: float = 2.0, width: int = 640,
                  height: int = 480, f: float = 525.0, dim: int = 512, vox: float = 0.01, stride: int = 4,
                  n_particles: int = 10240, iters: int = 20, mu: float = 0.15) -> Sequence:
    # the room fills the volume, leaving a 10 cm margin (5.02 m at 512^3 x 1 cm)
    scene = procedural_room(scene_seed, 0.1, dim * vox - 0.1)
    K = Intrinsics.centred(width, height, f * width / 640.0)
    poses = fast_trajectory(scene, traj_seed, n_frames, fps, speed, ang_speed)
    return Sequence(scene, K, (dim, dim, dim), vox, np.zeros(3), mu, poses, noise_seed, 0.002, 0.2, 6.0,
                    stride, n_particles, iters)


def _free_point(scene: Scene, rng, clearance: float) -> np.ndarray:
    lo, hi = scene.room_lo, scene.room_hi
    for _ in range(10000):
        p = rng.uniform(lo + clearance, hi - clearance)
        if scene.sdf(p[None])[0] >= clearance:
            return p
    raise RuntimeError("no free point")


def axis_motion(scene: Scene, seed: int, n_frames: int, fps: float, kind: str) -> List[Pose]:
    """Motions of the rescaling ablation's sequence sets.
    kind "1d": translation along, or rotation about, one camera axis (chosen
    by the seed), with the speed varying smoothly in [0.5, 4] m/s or
    [0.2, 5] rad/s; a translating camera turns back when it would come
    within 0.5 m of the room's boxes or walls.  kind "3d": rotation only,
    about a smoothly varying body axis at [0.2, 5] rad/s, from a fixed
    free-space point.  Every camera starts looking at the room centre."""
    rng = np.random.default_rng(seed)
    centre = 0.5 * (scene.room_lo + scene.room_hi)
    t = _free_point(scene, rng, 0.8)
    R = look_rotation(centre - t)
    dt = 1.0 / fps
    f1, p1 = rng.uniform(0.1, 0.5), rng.uniform(0, 2 * np.pi)
    axis = int(rng.integers(3))
    translate = kind == "1d" and bool(rng.integers(2))
    freqs = rng.uniform(0.05, 0.4, size=(3, 3))
    phases = rng.uniform(0, 2 * np.pi, size=(3, 3))
    sign = 1.0
    poses = []
    for k in range(n_frames):
        poses.append(Pose(R.copy(), t.copy()))
        tk = k * dt
        level = 0.5 + 0.5 * np.sin(2 * np.pi * f1 * tk + p1)
        if translate:
            v = 0.5 + 3.5 * level
            d = R[:, axis] * sign
            nxt = t + v * dt * d
            if scene.sdf(nxt[None])[0] < 0.5 or np.any(nxt < scene.room_lo + 0.5) or np.any(nxt > scene.room_hi - 0.5):
                sign = -sign
                nxt = t - v * dt * d
            t = nxt
        else:
            w = 0.2 + 4.8 * level
            if kind == "1d":
                a = np.zeros(3)
                a[axis] = 1.0
            else:
                a = np.array([np.sum(np.sin(2 * np.pi * freqs[d] * tk + phases[d])) for d in range(3)])
                a = a / max(np.linalg.norm(a), 1e-9)
            R = R @ axis_angle(a, w * dt)
            U, _, Vt = np.linalg.svd(R)
            R = U @ Vt
    return poses


def ablation_sequence(kind: str, seed: int, n_frames: int = 60, width: int = 320, height: int = 240,
                      dim: int = 512, vox: float = 0.01, mu: float = 0.15) -> Sequence:
    """A sequence of the ablation sets: kind "1d", "3d" (axis_motion),
    "6d" (fast_trajectory at a seeded speed in [1, 4] m/s and 0.67 x that in
    rad/s) or "6dfast" (the same at [4, 8] m/s), in a procedural room filling
    the volume, 320x240 depth."""
    scene = procedural_room(seed, 0.1, dim * vox - 0.1)
    K = Intrinsics.centred(width, height, 525.0 * width / 640.0)
    if kind in ("6d", "6dfast"):
        lo, hi = (1.0, 4.0) if kind == "6d" else (4.0, 8.0)
        v = float(np.random.default_rng(seed).uniform(lo, hi))
        poses = fast_trajectory(scene, seed + 1, n_frames, 30.0, v, 0.67 * v)
    else:
        poses = axis_motion(scene, seed + 1, n_frames, 30.0, kind)
    return Sequence(scene, K, (dim, dim, dim), vox, np.zeros(3), mu, poses, seed + 2, 0.002, 0.2, 6.0, 4, 10240, 20)
