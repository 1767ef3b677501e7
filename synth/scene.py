"""Analytic scenes: signed distance fields and closed-form ray casting.

Seeded input generation only -- nothing here computes a step of the pose
search or of the fusion.  Scenes stand in for the paper's indoor datasets
(ICL-NUIM, FastCaMo-Synth built on Replica, Sec. 5.1), which are not used.

Conventions
-----------
* World frame: metres, z up.
* Free-space signed distance: positive in free space, negative inside solid.
* A scene is a room interior (an axis-aligned box whose walls are solid on the
  outside) plus obstacles: spheres, axis-aligned boxes and vertical capped
  cylinders.
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np


@dataclasses.dataclass
class Sphere:
    c: np.ndarray  # (3,)
    r: float


@dataclasses.dataclass
class Box:
    lo: np.ndarray  # (3,)
    hi: np.ndarray  # (3,)


@dataclasses.dataclass
class Cylinder:
    """Vertical (z-axis) capped cylinder."""
    cx: float
    cy: float
    z0: float
    z1: float
    r: float


@dataclasses.dataclass
class Scene:
    room_lo: np.ndarray
    room_hi: np.ndarray
    spheres: List[Sphere] = dataclasses.field(default_factory=list)
    boxes: List[Box] = dataclasses.field(default_factory=list)
    cylinders: List[Cylinder] = dataclasses.field(default_factory=list)

    # ------------------------------------------------------------------ SDF
    def sdf(self, X: np.ndarray) -> np.ndarray:
        """Free-space signed distance at points X (..., 3), float64."""
        X = np.asarray(X, dtype=np.float64)
        d = np.minimum(X - self.room_lo, self.room_hi - X).min(axis=-1)
        for s in self.spheres:
            d = np.minimum(d, np.linalg.norm(X - s.c, axis=-1) - s.r)
        for b in self.boxes:
            c = 0.5 * (b.lo + b.hi)
            h = 0.5 * (b.hi - b.lo)
            q = np.abs(X - c) - h
            outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
            inside = np.minimum(q.max(axis=-1), 0.0)
            d = np.minimum(d, outside + inside)
        for cy in self.cylinders:
            rad = np.hypot(X[..., 0] - cy.cx, X[..., 1] - cy.cy) - cy.r
            zc = 0.5 * (cy.z0 + cy.z1)
            hz = np.abs(X[..., 2] - zc) - 0.5 * (cy.z1 - cy.z0)
            q = np.stack([rad, hz], axis=-1)
            outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
            inside = np.minimum(q.max(axis=-1), 0.0)
            d = np.minimum(d, outside + inside)
        return d

    # -------------------------------------------------------------- raycast
    def raycast(self, o: np.ndarray, d: np.ndarray) -> np.ndarray:
        """Smallest positive ray parameter t with o + t d on a surface.

        o: (3,) ray origin; d: (n, 3) directions (not normalised).  Returns
        (n,) float64, +inf where nothing is hit.
        """
        o = np.asarray(o, dtype=np.float64)
        d = np.asarray(d, dtype=np.float64)
        n = d.shape[0]
        t = np.full(n, np.inf)
        with np.errstate(divide="ignore", invalid="ignore"):
            # room interior: exit distance through the walls
            for a in range(3):
                da = d[:, a]
                ta = np.where(da > 0, (self.room_hi[a] - o[a]) / da,
                              np.where(da < 0, (self.room_lo[a] - o[a]) / da, np.inf))
                ta = np.where(ta > 0, ta, np.inf)
                t = np.minimum(t, ta)
            # dot products written out (no BLAS: its rounding may depend on threading)
            dd = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
            for s in self.spheres:
                oc = o - s.c
                b = d[:, 0] * oc[0] + d[:, 1] * oc[1] + d[:, 2] * oc[2]
                cc = oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2] - s.r * s.r
                disc = b * b - dd * cc
                sq = np.sqrt(np.maximum(disc, 0.0))
                t0 = (-b - sq) / dd
                t1 = (-b + sq) / dd
                th = np.where(t0 > 1e-9, t0, np.where(t1 > 1e-9, t1, np.inf))
                th = np.where(disc >= 0, th, np.inf)
                t = np.minimum(t, th)
            for bx in self.boxes:
                tn = np.full(n, -np.inf)
                tf = np.full(n, np.inf)
                for a in range(3):
                    da = d[:, a]
                    t_lo = (bx.lo[a] - o[a]) / da
                    t_hi = (bx.hi[a] - o[a]) / da
                    lo = np.minimum(t_lo, t_hi)
                    hi = np.maximum(t_lo, t_hi)
                    par = da == 0
                    inside_slab = (o[a] >= bx.lo[a]) & (o[a] <= bx.hi[a])
                    lo = np.where(par, np.where(inside_slab, -np.inf, np.inf), lo)
                    hi = np.where(par, np.where(inside_slab, np.inf, -np.inf), hi)
                    tn = np.maximum(tn, lo)
                    tf = np.minimum(tf, hi)
                hit = (tn <= tf) & (tf > 1e-9)
                th = np.where(hit, np.where(tn > 1e-9, tn, tf), np.inf)
                t = np.minimum(t, th)
            for cy in self.cylinders:
                ox, oy = o[0] - cy.cx, o[1] - cy.cy
                a2 = d[:, 0] ** 2 + d[:, 1] ** 2
                b2 = ox * d[:, 0] + oy * d[:, 1]
                c2 = ox * ox + oy * oy - cy.r * cy.r
                disc = b2 * b2 - a2 * c2
                sq = np.sqrt(np.maximum(disc, 0.0))
                best = np.full(n, np.inf)
                for sgn in (-1.0, 1.0):
                    ts = (-b2 + sgn * sq) / a2
                    z = o[2] + ts * d[:, 2]
                    ok = (disc >= 0) & (a2 > 0) & (ts > 1e-9) & (z >= cy.z0) & (z <= cy.z1)
                    best = np.minimum(best, np.where(ok, ts, np.inf))
                for zc in (cy.z0, cy.z1):
                    ts = (zc - o[2]) / d[:, 2]
                    px = ox + ts * d[:, 0]
                    py = oy + ts * d[:, 1]
                    ok = (d[:, 2] != 0) & (ts > 1e-9) & (px * px + py * py <= cy.r * cy.r)
                    best = np.minimum(best, np.where(ok, ts, np.inf))
                t = np.minimum(t, best)
        return t


# ---------------------------------------------------------------- builders
def unit_box_room(seed: int, n_spheres: int = 3) -> Scene:
    """Box room [-0.5, 0.5]^3 plus spheres of radius U(0.1, 0.3).

    Centres are rejection-sampled inside the room with a 2 cm margin,
    non-overlapping, and at least r + 0.15 m from the origin (where the
    cameras sit).
    """
    rng = np.random.default_rng(seed)
    lo = np.full(3, -0.5)
    hi = np.full(3, 0.5)
    spheres: List[Sphere] = []
    tries = 0
    while len(spheres) < n_spheres:
        tries += 1
        if tries > 100000:
            raise RuntimeError("sphere placement failed")
        r = rng.uniform(0.1, 0.3)
        c = rng.uniform(lo + 0.02, hi - 0.02)
        if np.linalg.norm(c) < r + 0.15:
            continue
        if any(np.linalg.norm(c - s.c) < r + s.r for s in spheres):
            continue
        spheres.append(Sphere(c, r))
    return Scene(lo, hi, spheres=spheres)


def procedural_room(seed: int, lo: float = 0.1, hi: float = 5.02) -> Scene:
    """Room interior [lo, hi]^3 with 6-10 boxes (edges 0.2-1.0 m) resting on
    the floor, 3-6 vertical cylinders (r 0.1-0.3, h 0.5-2.0) standing on the
    floor and 3-6 floating spheres (r 0.1-0.4)."""
    rng = np.random.default_rng(seed)
    rlo = np.full(3, lo)
    rhi = np.full(3, hi)
    sc = Scene(rlo, rhi)
    span = hi - lo
    for _ in range(int(rng.integers(6, 11))):
        e = rng.uniform(0.2, 1.0, size=3)
        xy = rng.uniform(lo + 0.05, hi - 0.05 - e[:2])
        blo = np.array([xy[0], xy[1], lo])
        sc.boxes.append(Box(blo, blo + e))
    for _ in range(int(rng.integers(3, 7))):
        r = rng.uniform(0.1, 0.3)
        h = rng.uniform(0.5, 2.0)
        c = rng.uniform(lo + r + 0.05, hi - r - 0.05, size=2)
        sc.cylinders.append(Cylinder(float(c[0]), float(c[1]), lo, lo + h, r))
    for _ in range(int(rng.integers(3, 7))):
        r = rng.uniform(0.1, 0.4)
        c = rng.uniform(lo + r + 0.05, hi - r - 0.05, size=3)
        c[2] = rng.uniform(lo + 0.3 * span, hi - r - 0.05)
        sc.spheres.append(Sphere(c, r))
    return sc


def analytic_tsdf(scene: Scene, dims: Tuple[int, int, int], vox: float, origin, mu: float) -> np.ndarray:
    """The exact normalised TSDF of the scene sampled at voxel centres:
    clamp(sdf / mu, -1, 1), float32, linear layout [k][j][i]."""
    nx, ny, nz = dims
    o = np.asarray(origin, dtype=np.float64)
    xs = o[0] + (np.arange(nx) + 0.5) * vox
    ys = o[1] + (np.arange(ny) + 0.5) * vox
    zs = o[2] + (np.arange(nz) + 0.5) * vox
    out = np.empty((nz, ny, nx), dtype=np.float32)
    XX, YY = np.meshgrid(xs, ys, indexing="xy")
    for k, z in enumerate(zs):
        P = np.stack([XX, YY, np.full_like(XX, z)], axis=-1)
        out[k] = np.clip(scene.sdf(P) / mu, -1.0, 1.0).astype(np.float32)
    return out
