"""Batched tracking benchmark: many independent synthetic sequences of
uneven sizes tracked in lockstep through one persistent fitness launch per
iteration, captured in a HIP graph (pso_batch_*), against the same sequences
tracked one after another through the single-sequence path.

Sequences (seeds 1000 + i): TSDF 256^3 / 384^3 / 512^3 at 1 cm (the room
scaled to the volume), depth 320x240 (f = 262.5) or 640x480 (f = 525),
4096-16384 particles, 1-4 m/s with 0.67 x that in rad/s, stride 4, 20
iterations, fusion at the tracked pose after every frame.  Depth frames are
rendered on the host before timing and are resident in HBM.

The batch's fitness launch shape is chosen by timing the supported shapes
on the first frame steps (a small autotuner); the single-sequence path runs
in the switching mode.  Both paths give
bit-identical poses (tested); the JSON line reports frames/s and
evaluations/s of both and the ATE of every sequence.

Usage: python -m paper_2105_05600_amd.bench_batch [--sequences 32] [--frames 30]
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
from paper_2105_05600_amd import autotune, rose  # noqa: E402

DIMS = (256, 384, 512)
FRAMES = ((320, 240), (640, 480))
PARTICLES = (4096, 6144, 8192, 10240, 12288, 16384)


def log(msg):
    print(f"[bench_batch] {msg}", file=sys.stderr, flush=True)


def make_sequences(n, frames, small=False):
    """small: 128^3 volumes at 4 cm, 160x120 depth, 1024 particles, stride 3
    (work a single launch cannot spread over the whole GPU)."""
    seqs = []
    for i in range(n):
        rng = np.random.default_rng(1000 + i)
        v = float(rng.uniform(1.0, 4.0))
        if small:
            seqs.append(synth.room_sequence(scene_seed=1000 + i, traj_seed=2000 + i, noise_seed=3000 + i,
                                            n_frames=frames, speed=v, ang_speed=0.67 * v, width=160, height=120,
                                            dim=128, vox=0.04, stride=3, n_particles=1024))
            continue
        dim = int(rng.choice(DIMS))
        w, h = FRAMES[int(rng.integers(2))]
        npart = int(rng.choice(PARTICLES))
        seqs.append(synth.room_sequence(scene_seed=1000 + i, traj_seed=2000 + i, noise_seed=3000 + i,
                                        n_frames=frames, speed=v, ang_speed=0.67 * v, width=w, height=h,
                                        dim=dim, n_particles=npart))
    return seqs


def fresh(seqs, depths):
    """Volumes fused from frame 0 and states at frame 0's pose (r_1 = 0.55)."""
    vols, states = [], (rose.TrackState * len(seqs))()
    for i, sq in enumerate(seqs):
        vol = rose.Tsdf(sq.dims, sq.vox, sq.mu, sq.origin)
        p0 = sq.poses[0]
        vol.integrate(depths[i][0], sq.K, p0.q, p0.t)
        vols.append(vol)
        states[i] = rose.track_state(p0.q, p0.t, [0.55] * 6)
    return vols, states


def learned_comparison(n, frames, seed_base, modes=("plain_single", "plain_batched", "learned", "untrained",
                                                      "small_carried"), log=lambda s: None, single_shape=(0, 0),
                       batch_shape=(0, 0)):
    """The same n held-out 320x240 sequences (seeds seed_base + 10 i, 1-4
    m/s) tracked for `frames` frames, fused at the tracked pose, in each of
    the modes:
    * plain_single: plain PST (10240 particles, 20 iterations), one sequence
      after another through pso_track_frame;
    * plain_batched: the same budget, batched (pso_batch_track);
    * learned: the learned proposal batched (pso_batch_track_learned with the
      committed weights and settings: small template and iteration count,
      per-sequence plain fallback);
    * untrained: the same path with an untrained network of the same shape;
    * small_carried: the learned run's budget batched, centre and axis
      lengths carried from the previous frame (no network).
    The single-sequence path runs in single_shape, the batched modes in
    batch_shape (both the switching mode by default: a batched sequence with
    2^23 or more evaluations per iteration, as every one here, then takes
    the single path's own launches inside the batch).  Returns {mode:
    {"frames_per_s", "ate_rmse_m" (per sequence), "ate_rmse_mean_m",
    "ate_rmse_median_m", "fallbacks"}}."""
    from paper_2105_05600_amd import train_proposal as tp
    import synth.mlp_init as mlp_init
    weights = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "proposal.npz")
    with open(os.path.splitext(weights)[0] + ".json") as f:
        meta = json.load(f)
    seqs = [tp.make_sequence(seed_base + 10 * i, frames, 320, 240) for i in range(n)]
    t0 = time.perf_counter()
    depths = [[torch.from_numpy(d).cuda() for d in sq.depths(range(frames), workers=16)] for sq in seqs]
    log(f"rendered {n} x {frames} frames in {time.perf_counter() - t0:.1f} s")
    net = rose.Mlp(tp.FEATURE_DIM, 256, 12, max_batch=max(64, n))
    trained = net.pack(tp.load(weights))
    untrained = net.pack(mlp_init.init_params(1))
    iters = meta.get("iters", 0) or 20
    pst_small = rose.pst_sample(meta.get("particles", 4096), 5600)
    pst_plain = rose.pst_sample(10240, 5600)
    plain = rose.track_params(max_iters=20, stride=4)
    small = rose.track_params(max_iters=iters, stride=4)
    lp = rose.learned_params(scale=8, kappa=meta["kappa"], delta=meta["delta"], iters=iters)
    steps = n * (frames - 1)
    out = {}
    for mode in modes:
        rose.set_fitness_shape(*(single_shape if mode == "plain_single" else batch_shape))
        vols, states = [], (rose.TrackState * n)()
        for i, sq in enumerate(seqs):
            vol = rose.Tsdf(sq.dims, sq.vox, sq.mu, sq.origin)
            p0 = sq.poses[0]
            vol.integrate(depths[i][0], sq.K, p0.q, p0.t)
            vols.append(vol)
            states[i] = rose.track_state(p0.q, p0.t, [0.55] * 6)
        est = [[np.array(sq.poses[0].t)] for sq in seqs]
        b = None
        if mode == "plain_batched":
            b = rose.Batch(vols, [sq.K for sq in seqs], [pst_plain] * n, [plain] * n, use_graph=True)
        elif mode != "plain_single":
            b = rose.Batch(vols, [sq.K for sq in seqs], [pst_small] * n, [small] * n,
                           use_graph=(mode == "small_carried"))
        work = torch.zeros(n * (tp.LOW_W * tp.LOW_H + tp.FEATURE_DIM + 12), device="cuda")
        vel = [[0.0] * 6 for _ in range(n)]
        fallbacks = 0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for f in range(1, frames):
            if mode == "plain_single":
                for i, sq in enumerate(seqs):
                    r = rose.track_frame(vols[i], depths[i][f], sq.K, pst_plain, plain, states[i])
                    est[i].append(np.array(r["t"]))
                    vols[i].integrate(depths[i][f], sq.K, r["q"], r["t"])
                continue
            prev = [(list(states[i].pose.q), list(states[i].pose.t)) for i in range(n)]
            if mode in ("learned", "untrained"):
                res = rose.batch_track_learned(b, [d[f] for d in depths], net,
                                               trained if mode == "learned" else untrained, work, vel, lp,
                                               [pst_plain] * n, [plain] * n, states)
                fallbacks += sum(int(r["fallback"]) for r in res)
            else:
                b.track([d[f] for d in depths], states)
            for i, sq in enumerate(seqs):
                q, t = list(states[i].pose.q), list(states[i].pose.t)
                vel[i] = rose.chart_log(prev[i][0], prev[i][1], q, t)
                est[i].append(np.array(t))
                vols[i].integrate(depths[i][f], sq.K, q, t)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        if b is not None:
            b.close()
        for v in vols:
            v.close()
        ates = [synth.ate(np.array(e), np.array([p.t for p in sq.poses[:frames]]))[1] for e, sq in zip(est, seqs)]
        out[mode] = {"frames_per_s": steps / wall, "ate_rmse_m": ates, "ate_rmse_mean_m": float(np.mean(ates)),
                     "ate_rmse_median_m": float(np.median(ates)), "fallbacks": fallbacks}
        log(f"{mode}: {steps / wall:.1f} frames/s, ATE mean {np.mean(ates):.4f} m, median {np.median(ates):.4f} m, "
            f"fallbacks {fallbacks}")
    rose.set_fitness_shape(4, 2)
    return out


def learned_main(args):
    """Plain PST one sequence after another and batched, the learned proposal
    batched with the trained and with an untrained network, and the learned
    run's budget without a network, on the same held-out 320x240 sequences
    (see learned_comparison)."""
    res = learned_comparison(args.sequences, args.frames, args.seed_base, log=log,
                             batch_shape=tuple(args.batch_shape))
    out = {"metric": "learned proposal batched vs plain PST: frames/s over all sequences and ATE",
           "sequences": args.sequences, "frames": args.frames, "image": [320, 240], "seed_base": args.seed_base}
    for mode, r in res.items():
        out[mode] = {k: v for k, v in r.items()}
    out["speedup_learned_vs_plain_single"] = res["learned"]["frames_per_s"] / res["plain_single"]["frames_per_s"]
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sequences", type=int, default=32)
    ap.add_argument("--frames", type=int, default=30)
    ap.add_argument("--tune-steps", type=int, default=3)
    ap.add_argument("--small", action="store_true", help="small sequences (128^3 at 4 cm, 160x120, 1024 particles)")
    ap.add_argument("--seed-base", type=int, default=52000, help="--learned: first sequence seed")
    ap.add_argument("--batch-shape", type=int, nargs=2, default=[0, 0],
                    help="--learned: fitness launch shape of the batched modes ((0, 0): switching mode)")
    ap.add_argument("--learned", action="store_true",
                    help="learned proposal, batched, against plain PST one sequence after another (320x240)")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    if args.learned:
        return learned_main(args)
    seqs = make_sequences(args.sequences, args.frames, args.small)
    t0 = time.perf_counter()
    depths = [[torch.from_numpy(d).cuda() for d in sq.depths(range(args.frames), workers=16)] for sq in seqs]
    log(f"rendered {args.sequences} x {args.frames} frames in {time.perf_counter() - t0:.1f} s")
    psts = {n: rose.pst_sample(n, 5600) for n in sorted({sq.n_particles for sq in seqs})}
    params = [rose.track_params(max_iters=sq.iters, stride=sq.stride) for sq in seqs]
    stream = torch.cuda.Stream()

    # launch-shape tuning: time a few frame steps of the batch per shape
    tune_ms = {}
    for shape in autotune.BATCH_SHAPES:
        rose.set_fitness_shape(*shape)
        vols, states = fresh(seqs, depths)
        with torch.cuda.stream(stream):
            b = rose.Batch(vols, [sq.K for sq in seqs], [psts[sq.n_particles] for sq in seqs], params)
            b.track([d[1] for d in depths], states, stream=stream)  # capture
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for f in range(2, 2 + args.tune_steps):
                b.track([d[f] for d in depths], states, stream=stream)
            torch.cuda.synchronize()
        tune_ms[f"{shape[0]}x{shape[1]}"] = 1e3 * (time.perf_counter() - t1) / args.tune_steps
        b.close()
        for v in vols:
            v.close()
    best = min(autotune.BATCH_SHAPES, key=lambda s: tune_ms[f"{s[0]}x{s[1]}"])
    rose.set_fitness_shape(*best)
    log(f"batch shape {best} (ms per frame step: {tune_ms})")

    # batched run (graph-captured)
    vols, states = fresh(seqs, depths)
    est_b = [[np.array(sq.poses[0].t)] for sq in seqs]
    evals = 0.0
    with torch.cuda.stream(stream):
        b = rose.Batch(vols, [sq.K for sq in seqs], [psts[sq.n_particles] for sq in seqs], params)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for f in range(1, args.frames):
            res = b.track([d[f] for d in depths], states, stream=stream)
            for i, sq in enumerate(seqs):
                evals += sq.n_particles * float(sum(res[i]["n_overlap"]))
                est_b[i].append(np.array(res[i]["t"]))
                vols[i].integrate(depths[i][f], sq.K, res[i]["q"], res[i]["t"], stream=stream)
        torch.cuda.synchronize()
        wall_b = time.perf_counter() - t1
    b.close()
    for v in vols:
        v.close()

    # the same sequences through the single-sequence path, one after another,
    # in its own default launch configuration (the switching mode)
    rose.set_fitness_shape(0, 0)
    vols, states = fresh(seqs, depths)
    est_s = [[np.array(sq.poses[0].t)] for sq in seqs]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for f in range(1, args.frames):
        for i, sq in enumerate(seqs):
            r = rose.track_frame(vols[i], depths[i][f], sq.K, psts[sq.n_particles], params[i], states[i])
            est_s[i].append(np.array(r["t"]))
            vols[i].integrate(depths[i][f], sq.K, r["q"], r["t"])
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t1
    for v in vols:
        v.close()

    same = all(np.array_equal(np.array(a), np.array(c)) for a, c in zip(est_b, est_s))
    ates = [synth.ate(np.array(e), np.array([p.t for p in sq.poses[:args.frames]]))[1] for e, sq in zip(est_b, seqs)]
    steps = args.sequences * (args.frames - 1)
    out = {"metric": "batched tracking: frames/s and particle*point evals/s over all sequences",
           "sequences": args.sequences, "frames": args.frames, "small": args.small,
           "config": [{"tsdf": sq.dims[0], "image": [sq.K.width, sq.K.height], "particles": sq.n_particles}
                      for sq in seqs],
           "shape": list(best), "tune_ms_per_step": tune_ms,
           "batch": {"wall_s": wall_b, "frames_per_s": steps / wall_b, "evals_per_s": evals / wall_b},
           "single": {"wall_s": wall_s, "frames_per_s": steps / wall_s, "evals_per_s": evals / wall_s},
           "speedup": wall_s / wall_b, "poses_identical": bool(same),
           "ate_rmse_m": {"mean": float(np.mean(ates)), "max": float(np.max(ates)), "per_sequence": ates}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
