"""Trajectory metrics of Sec. 5.1.

* ATE: the estimated trajectory is rigidly aligned to the ground truth
  (Horn's closed-form absolute orientation, no scale), then the translation
  differences are averaged; both the mean and the RMSE are returned.
* TE (Eq. te): || trans( T_G^-1 T_E ) ||_2 per frame, no pre-alignment.
"""
from __future__ import annotations

import numpy as np


def horn_align(src: np.ndarray, dst: np.ndarray):
    """Rigid (R, t) minimising sum ||R src_i + t - dst_i||^2 (no scale),
    via the SVD form of Horn / Umeyama."""
    src = np.asarray(src, dtype=np.float64)
    dst = np.asarray(dst, dtype=np.float64)
    ms, md = src.mean(0), dst.mean(0)
    H = (src - ms).T @ (dst - md)
    U, _, Vt = np.linalg.svd(H)
    D = np.eye(3)
    D[2, 2] = np.sign(np.linalg.det(Vt.T @ U.T))
    R = Vt.T @ D @ U.T
    t = md - R @ ms
    return R, t


def ate(est_t: np.ndarray, gt_t: np.ndarray):
    """(mean, rmse) of translation error after rigid alignment of est to gt."""
    est_t = np.asarray(est_t, dtype=np.float64)
    gt_t = np.asarray(gt_t, dtype=np.float64)
    if len(est_t) < 3:
        e = np.linalg.norm(est_t - gt_t, axis=1)
    else:
        R, t = horn_align(est_t, gt_t)
        e = np.linalg.norm(est_t @ R.T + t - gt_t, axis=1)
    return float(e.mean()), float(np.sqrt((e * e).mean()))


def translation_error(T_gt: np.ndarray, T_est: np.ndarray) -> float:
    """Eq. te: translation part of T_G^-1 T_E (4x4 homogeneous matrices)."""
    D = np.linalg.inv(np.asarray(T_gt)) @ np.asarray(T_est)
    return float(np.linalg.norm(D[:3, 3]))
