"""Ablation experiments of the paper's Sec. 5 on synthetic sequences, run
through the library (one GPU).

  rescale   Fig. "ablation of rescaling": PST rescaling with both parts of
            Eq. rsinter, with the isotropic part only and with the
            anisotropic part only, on three sets of sequences -- motion along
            or about one camera axis (0.5-4 m/s, 0.2-5 rad/s), pure 3D
            rotation (0.2-5 rad/s) and 6D motion (1-4 m/s).  Reported: the
            average fitness (rho~ of Eq. wafit; the threshold when the APS is
            empty) at every iteration over all frames, with its 10th and
            90th percentiles.
  tsdf      Tab. "TSDF normalisation": the fitness with and without the
            overlap set O_k (Eq. validness), with and without the
            normalisation of Eq. normallh, and with plain binary32 sums
            instead of compensated ones ("No Kahan"); ATE on the 6D set.
  multires  Fig. "multi-resolution": the alternating (1024, 1/8),
            (3072, 1/16), (10240, 1/32) schedule (strides 3, 4, 6) against
            each single setting and the 10240-particle stride-4 default;
            ATE and tracking time per frame on the 6D set.
  template  i.i.d. uniform template vs the 6D Poisson-disk template (Sec. 4
            "PST pre-sampling"); ATE and time per frame on the 6D set.
  optimizer Fig. "optimisation strategy": PFO with PST against vanilla PFO
            (Gaussian proposal + resampling, Eq. pfolh) and PSO (inertia
            weight 0.9 -> 0.4, c1 = c2 = 2), all with 10240 particles, 20
            iterations and the fitness of Eq. normallh, on the 6D set and on
            a faster 6D set (4-8 m/s, 2.7-5.4 rad/s).
            PFO with PST also runs with the centre's exact fitness as the
            APS threshold.  Reported per iteration: the exact fitness of each method's
            current estimate (PST: the centre c_k; the others: the best state
            so far) averaged over all frames, with its percentiles; ATE and
            time per frame.  The comparison methods have no adaptive scale:
            they run at three initial spreads r_init (sigma = r_init/sqrt8,
            vmax = r_init).

Every sequence is tracked frame by frame (20 iterations, fusion at the
tracked pose) from its first ground-truth pose.  ATE: translation RMSE after
Horn alignment.  320x240 depth (f = 262.5), 512^3 TSDF at 1 cm, mu = 15 cm.

Usage: python -m paper_2105_05600_amd.ablation --out results.json \\
           [--experiments rescale,tsdf,multires,template,optimizer] [--sequences 10]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from paper_2105_05600_amd import rose  # noqa: E402

ITERS = 20
MULTIRES = [(1024, 3), (3072, 4), (10240, 6)]


def log(msg):
    print(f"[ablation] {msg}", flush=True)


def track(sq, depths, pst, params):
    """Track a sequence; returns (ATE RMSE, ms per frame of the tracking
    calls, per-frame rho~ per iteration)."""
    vol = rose.Tsdf(sq.dims, sq.vox, sq.mu, sq.origin)
    p0 = sq.poses[0]
    st = rose.track_state(p0.q, p0.t, [1.0] * 6, tsdf_built=False)
    rose.track_frame(vol, depths[0], sq.K, pst, params, st)
    vol.integrate(depths[0], sq.K, p0.q, p0.t)
    st.tsdf_built = 1
    est = [np.array(p0.t)]
    rho = []
    t_track = 0.0
    for f in range(1, len(depths)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            r = rose.track_frame(vol, depths[f], sq.K, pst, params, st)
        except rose.RoseError as e:  # a frame without valid depth: the pose is kept
            if e.status != rose.E_STATE:
                raise
            r = None
        t_track += time.perf_counter() - t0
        if r is not None:
            rho.append(r["rho_iter"] + [r["rho_iter"][-1]] * (ITERS - len(r["rho_iter"])))
        est.append(np.array(st.pose.t))
        vol.integrate(depths[f], sq.K, st.pose.q, st.pose.t)
    vol.close()
    gt = np.array([p.t for p in sq.poses[:len(depths)]])
    _, rmse = synth.ate(np.array(est), gt)
    return float(rmse), 1e3 * t_track / (len(depths) - 1), rho


def track_pst_curve(sq, depths, pst, flags=0):
    """PFO with PST (20 iterations) with the exact fitness of the centre c_k
    after every iteration k: a 21-iteration run from a copy of the state
    reads rho(c_k) as particle 0's fitness of iteration k + 1 (the first 20
    iterations of both runs are the same computation)."""
    params = rose.track_params(max_iters=ITERS, stride=4, flags=flags)
    probe_params = rose.track_params(max_iters=ITERS + 1, stride=4, flags=flags)
    vol = rose.Tsdf(sq.dims, sq.vox, sq.mu, sq.origin)
    p0 = sq.poses[0]
    st = rose.track_state(p0.q, p0.t, [1.0] * 6, tsdf_built=False)
    rose.track_frame(vol, depths[0], sq.K, pst, params, st)
    vol.integrate(depths[0], sq.K, p0.q, p0.t)
    st.tsdf_built = 1
    est, curves, t_track = [np.array(p0.t)], [], 0.0
    for f in range(1, len(depths)):
        probe = rose.track_state(list(st.pose.q), list(st.pose.t), list(st.r))
        try:
            r = rose.track_frame(vol, depths[f], sq.K, pst, probe_params, probe)
            curves.append(r["rho_centre"][1:ITERS + 1])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rose.track_frame(vol, depths[f], sq.K, pst, params, st)
            t_track += time.perf_counter() - t0
        except rose.RoseError as e:  # a frame without valid depth: the pose is kept
            if e.status != rose.E_STATE:
                raise
        est.append(np.array(st.pose.t))
        vol.integrate(depths[f], sq.K, st.pose.q, st.pose.t)
    vol.close()
    gt = np.array([p.t for p in sq.poses[:len(depths)]])
    _, rmse = synth.ate(np.array(est), gt)
    return float(rmse), 1e3 * t_track / (len(depths) - 1), curves


def track_swarm(sq, depths, pst, method, params, seed):
    """Vanilla PFO or PSO frame by frame (random draws from a seeded torch
    generator on the GPU, drawn outside the timed calls); returns (ATE RMSE,
    ms per frame, per-frame rho of the best state after every iteration)."""
    vol = rose.Tsdf(sq.dims, sq.vox, sq.mu, sq.origin)
    p0 = sq.poses[0]
    st = rose.track_state(p0.q, p0.t, [1.0] * 6)
    vol.integrate(depths[0], sq.K, p0.q, p0.t)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    n = pst.shape[0]
    est, curves, t_track = [np.array(p0.t)], [], 0.0
    for f in range(1, len(depths)):
        if method == rose.PFO:
            draws = torch.randn((ITERS, n, 6), generator=gen, device="cuda")
            offsets = torch.rand(ITERS, generator=gen, device="cuda")
        else:
            draws = torch.rand((ITERS, n, 12), generator=gen, device="cuda")
            offsets = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            r = rose.swarm_track_frame(method, vol, depths[f], sq.K, pst, params, st, draws, offsets)
            curves.append(r["rho_best"])
        except rose.RoseError as e:
            if e.status != rose.E_STATE:
                raise
        t_track += time.perf_counter() - t0
        est.append(np.array(st.pose.t))
        vol.integrate(depths[f], sq.K, st.pose.q, st.pose.t)
    vol.close()
    gt = np.array([p.t for p in sq.poses[:len(depths)]])
    _, rmse = synth.ate(np.array(est), gt)
    return float(rmse), 1e3 * t_track / (len(depths) - 1), curves


def exp_optimizer(n_seq, frames, pst, base, kind="6d", spreads=(0.05, 0.1, 0.2)):
    runs = {"pfo_pst": None, "pfo_pst_centre_threshold": rose.FLAG_CENTRE_THRESHOLD}
    for r0 in spreads:
        runs[f"vanilla_pfo_r{r0}"] = (rose.PFO, r0)
        runs[f"pso_r{r0}"] = (rose.PSO, r0)
    rows = {v: {"ate": [], "ms": [], "curves": []} for v in runs}
    for seed, sq, depths in sequences(kind, n_seq, frames, base):
        for v, spec in runs.items():
            if spec is None or isinstance(spec, int):
                ate, ms, cv = track_pst_curve(sq, depths, pst, flags=spec or 0)
            else:
                method, r0 = spec
                params = rose.swarm_params(iters=ITERS, stride=4, r_init=(r0,) * 6)
                ate, ms, cv = track_swarm(sq, depths, pst, method, params, seed * 7 + method)
            rows[v]["ate"].append(ate)
            rows[v]["ms"].append(ms)
            rows[v]["curves"].extend(cv)
    res = {}
    for v, r in rows.items():
        a = np.array(r["curves"])  # frames x iterations
        res[v] = {"ate_rmse_mean_m": float(np.mean(r["ate"])), "ate_rmse_median_m": float(np.median(r["ate"])),
                  "ms_per_frame": float(np.mean(r["ms"])), "ate_per_sequence": r["ate"],
                  "rho_mean": a.mean(0).tolist(), "rho_p10": np.percentile(a, 10, axis=0).tolist(),
                  "rho_p25": np.percentile(a, 25, axis=0).tolist(), "rho_p75": np.percentile(a, 75, axis=0).tolist(),
                  "rho_p90": np.percentile(a, 90, axis=0).tolist(), "rho_min": a.min(0).tolist(),
                  "rho_max": a.max(0).tolist()}
        m = res[v]["rho_mean"]
        log(f"optimizer {kind} {v}: rho at iterations 1/2/5/10/20 {m[0]:.4f} {m[1]:.4f} {m[4]:.4f} {m[9]:.4f} {m[19]:.4f}; "
            f"ATE mean {res[v]['ate_rmse_mean_m']:.4f} m median {res[v]['ate_rmse_median_m']:.4f} m, "
            f"{res[v]['ms_per_frame']:.2f} ms/frame")
    return res


def sequences(kind, n, frames, base):
    for i in range(n):
        sq = synth.configs.ablation_sequence(kind, base + 10 * i, frames)
        yield base + 10 * i, sq, [torch.from_numpy(d).cuda() for d in sq.depths(range(frames), workers=16)]


def exp_rescale(n_seq, frames, pst):
    out = {}
    variants = {"both": 0, "iso_only": rose.FLAG_ISO_ONLY, "aniso_only": rose.FLAG_ANISO_ONLY}
    for kind, base in (("1d", 61000), ("3d", 62000), ("6d", 63000)):
        curves = {v: [] for v in variants}
        ates = {v: [] for v in variants}
        for seed, sq, depths in sequences(kind, n_seq, frames, base):
            for v, flag in variants.items():
                ate, ms, rho = track(sq, depths, pst, rose.track_params(max_iters=ITERS, stride=4, flags=flag))
                curves[v].extend(rho)
                ates[v].append(ate)
        res = {}
        for v in variants:
            a = np.array(curves[v])  # frames x iterations
            res[v] = {"mean": a.mean(0).tolist(), "p10": np.percentile(a, 10, axis=0).tolist(),
                      "p90": np.percentile(a, 90, axis=0).tolist(), "ate_rmse_mean_m": float(np.mean(ates[v]))}
            log(f"rescale {kind} {v}: rho~ at iterations 1/5/10/20 "
                f"{res[v]['mean'][0]:.4f} {res[v]['mean'][4]:.4f} {res[v]['mean'][9]:.4f} {res[v]['mean'][19]:.4f}; "
                f"ATE {res[v]['ate_rmse_mean_m']:.4f} m")
        out[kind] = res
    return out


def exp_variants(n_seq, frames, variants, base):
    """variants: name -> (pst, params); returns per-variant ATE and time."""
    rows = {v: {"ate": [], "ms": []} for v in variants}
    for seed, sq, depths in sequences("6d", n_seq, frames, base):
        for v, (pst, params) in variants.items():
            ate, ms, _ = track(sq, depths, pst, params)
            rows[v]["ate"].append(ate)
            rows[v]["ms"].append(ms)
    res = {}
    for v, r in rows.items():
        res[v] = {"ate_rmse_mean_m": float(np.mean(r["ate"])), "ate_rmse_median_m": float(np.median(r["ate"])),
                  "ms_per_frame": float(np.mean(r["ms"])), "ate_per_sequence": r["ate"]}
        log(f"{v}: ATE mean {res[v]['ate_rmse_mean_m']:.4f} m median {res[v]['ate_rmse_median_m']:.4f} m, "
            f"{res[v]['ms_per_frame']:.2f} ms/frame")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--experiments", default="rescale,tsdf,multires,template,optimizer")
    ap.add_argument("--sequences", type=int, default=10)
    ap.add_argument("--frames", type=int, default=60)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    pst = rose.pst_sample(10240, 5600)
    exps = args.experiments.split(",")
    res = {"sequences": args.sequences, "frames": args.frames}
    if "rescale" in exps:
        res["rescale"] = exp_rescale(args.sequences, args.frames, pst)
    if "tsdf" in exps:
        res["tsdf"] = exp_variants(args.sequences, args.frames, {
            "full": (pst, rose.track_params(max_iters=ITERS, stride=4)),
            "no_overlap": (pst, rose.track_params(max_iters=ITERS, stride=4, flags=rose.FLAG_NO_OVERLAP)),
            "no_normalize": (pst, rose.track_params(max_iters=ITERS, stride=4, flags=rose.FLAG_NO_NORMALIZE)),
            "no_kahan": (pst, rose.track_params(max_iters=ITERS, stride=4, flags=rose.FLAG_NO_KAHAN)),
        }, 64000)
    if "multires" in exps:
        var = {"single_10240_s4": (pst, rose.track_params(max_iters=ITERS, stride=4)),
               "alternating": (pst, rose.track_params(max_iters=ITERS, levels=MULTIRES)),
               "alternating_centre_threshold": (pst, rose.track_params(max_iters=ITERS, levels=MULTIRES,
                                                                       flags=rose.FLAG_CENTRE_THRESHOLD)),
               "alternating_dense_first": (pst, rose.track_params(max_iters=ITERS, levels=MULTIRES[::-1])),
               "alternating_21_dense_last": (pst, rose.track_params(max_iters=ITERS + 1, levels=MULTIRES)),
               "single_10240_s4_centre_threshold": (pst, rose.track_params(max_iters=ITERS, stride=4,
                                                                           flags=rose.FLAG_CENTRE_THRESHOLD))}
        for n, s in MULTIRES:
            var[f"single_{n}_s{s}"] = (pst[:n].contiguous(), rose.track_params(max_iters=ITERS, stride=s))
        res["multires"] = exp_variants(args.sequences, args.frames, var, 65000)
    if "template" in exps:
        ppd, got, drawn = rose.pst_poisson(10240, 5600, rose.poisson_radius(10240), 1 << 22)
        assert got == 10240, (got, drawn)
        res["template"] = exp_variants(args.sequences, args.frames, {
            "iid": (pst, rose.track_params(max_iters=ITERS, stride=4)),
            "poisson": (ppd, rose.track_params(max_iters=ITERS, stride=4)),
        }, 66000)
    if "optimizer" in exps:
        res["optimizer"] = exp_optimizer(args.sequences, args.frames, pst, 67000)
        res["optimizer_fast"] = exp_optimizer(args.sequences, args.frames, pst, 68000, kind="6dfast")
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
