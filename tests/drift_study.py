"""Tracking drift on the 512^3 room sequence (640x480, stride 4, 10240
particles, 20 iterations), from the oracle alone.  Test infrastructure: it
runs the oracle, never the HIP path.

Three runs over the first K frames:
* closed loop, binary32 mode -- the benchmark's protocol (frame 0 sets r_1 =
  0.55 and is fused at its true pose; frame t is tracked from the estimate
  of frame t-1 and fused at its own estimate) in the arithmetic the GPU
  path mirrors;
* closed loop, binary64 mode -- the same protocol with every step in
  binary64 (fusion, unprojection, overlap, fitness, update);
* open loop, binary32 mode -- every frame fused at its true pose, frame t
  tracked from the true pose of frame t-1 (axis lengths carried as in the
  closed loop), so that each frame's error is the tracker's own, without the
  map's accumulated drift.

Per frame it prints the translation error |t_est - t_true| and the rotation
error, and for each run the ATE (mean and RMSE after rigid alignment, as
the benchmark reports it).

    python tests/drift_study.py --frames 26 --threads 8 --out FILE
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import os

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
import synth  # noqa: E402


def _rot_err(qa, qb) -> float:
    Ra, Rb = synth.quat_to_mat(qa), synth.quat_to_mat(qb)
    return math.acos(float(np.clip((np.trace(Ra.T @ Rb) - 1) / 2, -1, 1)))


def run(seq, depths, pst, prec: int, closed: bool, log) -> dict:
    nx, ny, nz = seq.dims
    psi = np.ones((nz, ny, nx), np.float32)
    wt = np.zeros_like(psi)
    p0 = seq.poses[0]
    kw = dict(max_iters=seq.iters, stride=seq.stride, lookup=oracle.NEAREST, prec=prec)
    # frame 0: no fitness (Sec. 4, first corner case); r_1 = 0.1 + 0.9 * 0.5
    o = oracle.track_frame(psi, seq.vox, seq.origin, depths[0], seq.K, pst, p0.q, p0.t, np.ones(6),
                           tsdf_built=False, **kw)
    r = np.asarray(o["r1"])
    oracle.integrate(psi, wt, seq.vox, seq.origin, seq.mu, depths[0], seq.K, p0.q, p0.t, prec=prec)
    q_est, t_est = np.asarray(p0.q), np.asarray(p0.t)
    est = [t_est.copy()]
    frames = []
    for i in range(1, len(depths)):
        prev = (q_est, t_est) if closed else (seq.poses[i - 1].q, seq.poses[i - 1].t)
        t0 = time.perf_counter()
        o = oracle.track_frame(psi, seq.vox, seq.origin, depths[i], seq.K, pst, prev[0], prev[1], r, **kw)
        r = np.asarray(o["r1"])
        q_est, t_est = np.asarray(o["q"]), np.asarray(o["t"])
        est.append(t_est.copy())
        fuse = (q_est, t_est) if closed else (seq.poses[i].q, seq.poses[i].t)
        oracle.integrate(psi, wt, seq.vox, seq.origin, seq.mu, depths[i], seq.K, fuse[0], fuse[1], prec=prec)
        gt = seq.poses[i]
        f = dict(frame=i, t_err_m=float(np.linalg.norm(t_est - gt.t)), r_err_rad=_rot_err(q_est, gt.q),
                 aps_last=int(o["aps"][-1]), rho=float(o["rho"]), n_points=int(o["n_points"]),
                 step_m=float(np.linalg.norm(gt.t - seq.poses[i - 1].t)),
                 step_rad=_rot_err(gt.q, seq.poses[i - 1].q), s=time.perf_counter() - t0)
        frames.append(f)
        log(json.dumps(f))
    gt_t = np.array([p.t for p in seq.poses[:len(depths)]])
    mean, rmse = synth.ate(np.array(est), gt_t)
    return dict(ate_mean_m=mean, ate_rmse_m=rmse, frames=frames, t_est=[list(map(float, t)) for t in est])


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=26)
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--runs", default="closed-f32,closed-f64,open-f32")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    oracle.build(force=False)
    seq = synth.room_sequence()
    depths = seq.depths(range(a.frames), workers=a.threads)
    pst, _ = oracle.pst_sample(seq.n_particles, 5600)
    out = {}

    def log(s):
        print(s, flush=True)

    with oracle.threads(a.threads):
        for name in a.runs.split(","):
            loop, mode = name.split("-")
            log(f"run {name}")
            out[name] = run(seq, depths, pst, oracle.F32 if mode == "f32" else oracle.F64, loop == "closed", log)
            log(f"{name}: ATE mean {out[name]['ate_mean_m']:.4f} m, RMSE {out[name]['ate_rmse_m']:.4f} m")
            with open(a.out, "w") as f:
                json.dump(out, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
