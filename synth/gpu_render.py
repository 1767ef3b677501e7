"""Depth rendering of the synthetic scenes with torch (binary64), batched over
frames: the same ray/primitive intersections as Scene.raycast (room walls,
spheres, axis-aligned boxes, vertical capped cylinders) and the same noise
model (z + N(0, (k z^2)^2), then (zmin, zmax) validity).  Used where many
frames are rendered on the GPU at once (training data for the learned
proposal); the noise comes from a seeded torch generator, so frames are not
bit-identical to the numpy renderer's noisy frames (noise-free frames agree
to rounding)."""
from __future__ import annotations

from typing import Sequence as Seq

import numpy as np
import torch

from .camera import Intrinsics, Pose, pixel_rays
from .scene import Scene

_INF = float("inf")


def _raycast(scene: Scene, o: torch.Tensor, d: torch.Tensor) -> torch.Tensor:
    """Smallest positive t with o + t d on a surface; o (F, 1, 3), d (F, N, 3)."""
    dev = d.device
    inf = torch.tensor(_INF, dtype=torch.float64, device=dev)
    lo = torch.as_tensor(scene.room_lo, dtype=torch.float64, device=dev)
    hi = torch.as_tensor(scene.room_hi, dtype=torch.float64, device=dev)
    t = torch.full(d.shape[:2], _INF, dtype=torch.float64, device=dev)
    for a in range(3):
        da = d[..., a]
        oa = o[..., a]
        ta = torch.where(da > 0, (hi[a] - oa) / da, torch.where(da < 0, (lo[a] - oa) / da, inf))
        t = torch.minimum(t, torch.where(ta > 0, ta, inf))
    dd = (d * d).sum(-1)
    for s in scene.spheres:
        oc = o - torch.as_tensor(s.c, dtype=torch.float64, device=dev)
        b = (d * oc).sum(-1)
        cc = (oc * oc).sum(-1) - s.r * s.r
        disc = b * b - dd * cc
        sq = torch.sqrt(torch.clamp(disc, min=0.0))
        t0 = (-b - sq) / dd
        t1 = (-b + sq) / dd
        th = torch.where(t0 > 1e-9, t0, torch.where(t1 > 1e-9, t1, inf))
        t = torch.minimum(t, torch.where(disc >= 0, th, inf))
    for bx in scene.boxes:
        tn = torch.full_like(t, -_INF)
        tf = torch.full_like(t, _INF)
        for a in range(3):
            da = d[..., a]
            oa = o[..., a]
            t_lo = (float(bx.lo[a]) - oa) / da
            t_hi = (float(bx.hi[a]) - oa) / da
            lo_a = torch.minimum(t_lo, t_hi)
            hi_a = torch.maximum(t_lo, t_hi)
            par = da == 0
            inside = (oa >= float(bx.lo[a])) & (oa <= float(bx.hi[a]))
            lo_a = torch.where(par, torch.where(inside, -inf, inf), lo_a)
            hi_a = torch.where(par, torch.where(inside, inf, -inf), hi_a)
            tn = torch.maximum(tn, lo_a)
            tf = torch.minimum(tf, hi_a)
        hit = (tn <= tf) & (tf > 1e-9)
        t = torch.minimum(t, torch.where(hit, torch.where(tn > 1e-9, tn, tf), inf))
    for cy in scene.cylinders:
        ox = o[..., 0] - cy.cx
        oy = o[..., 1] - cy.cy
        a2 = d[..., 0] ** 2 + d[..., 1] ** 2
        b2 = ox * d[..., 0] + oy * d[..., 1]
        c2 = ox * ox + oy * oy - cy.r * cy.r
        disc = b2 * b2 - a2 * c2
        sq = torch.sqrt(torch.clamp(disc, min=0.0))
        best = torch.full_like(t, _INF)
        for sgn in (-1.0, 1.0):
            ts = (-b2 + sgn * sq) / a2
            z = o[..., 2] + ts * d[..., 2]
            ok = (disc >= 0) & (a2 > 0) & (ts > 1e-9) & (z >= cy.z0) & (z <= cy.z1)
            best = torch.minimum(best, torch.where(ok, ts, inf))
        for zc in (cy.z0, cy.z1):
            ts = (zc - o[..., 2]) / d[..., 2]
            px = ox + ts * d[..., 0]
            py = oy + ts * d[..., 1]
            ok = (d[..., 2] != 0) & (ts > 1e-9) & (px * px + py * py <= cy.r * cy.r)
            best = torch.minimum(best, torch.where(ok, ts, inf))
        t = torch.minimum(t, best)
    return t


def render_depths(scene: Scene, K: Intrinsics, poses: Seq[Pose], zmin: float = 0.0, zmax: float = _INF,
                  noise_seed=None, noise_k: float = 0.0, device="cuda", frames_per_batch: int = 16) -> torch.Tensor:
    """(F, H, W) float32 z-depth of `poses` (rays with unit camera z, so the
    ray parameter is the z-depth).  With noise_k > 0, frame i gets
    N(0, (noise_k z^2)^2) noise from a torch generator seeded by
    (noise_seed, i)."""
    dc = torch.as_tensor(pixel_rays(K), dtype=torch.float64, device=device)  # (N, 3)
    out = torch.empty((len(poses), K.height, K.width), dtype=torch.float32, device=device)
    for f0 in range(0, len(poses), frames_per_batch):
        chunk = poses[f0:f0 + frames_per_batch]
        R = torch.as_tensor(np.stack([p.R for p in chunk]), dtype=torch.float64, device=device)
        o = torch.as_tensor(np.stack([p.t for p in chunk]), dtype=torch.float64, device=device)[:, None, :]
        d = dc[None] @ R.transpose(1, 2)
        z = _raycast(scene, o, d)
        if noise_k > 0:
            for k in range(len(chunk)):
                g = torch.Generator(device=device)
                base = 0 if noise_seed is None else int(noise_seed)
                g.manual_seed((base * 1_000_003 + f0 + k) & 0x7FFFFFFFFFFFFFFF)
                z[k] = z[k] + torch.randn(z[k].shape, generator=g, dtype=torch.float64, device=device) * noise_k * \
                    z[k] * z[k]
        z = torch.where(torch.isfinite(z) & (z > zmin) & (z < zmax), z, torch.zeros_like(z))
        out[f0:f0 + len(chunk)] = z.reshape(len(chunk), K.height, K.width).to(torch.float32)
    return out
