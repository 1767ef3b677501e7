"""Train the learned PST proposal on pairs produced by plain PST on the GPU,
then compare learned + fallback against plain PST on held-out sequences.

Data: seeded synthetic fast-motion sequences (procedural rooms, 320x240
depth with sigma = 0.002 z^2 noise, 1-4 m/s, angular speed 0.67 x linear
speed in rad/s).  Plain PST (10240 particles, 20 iterations) tracks every
sequence frame by frame -- many sequences at once through the batched
tracker -- and each frame t >= 2 yields one training pair:
  input  x_t: 40x30 depth residual of frame t against the model rendered at
              the plain result for t-1, plus the previous increment u_{t-1}
              (chart of Sec. 3.3), zero-padded to 1216;
  target y_t: the plain result's increment u_t = chart(s_{t-1}^-1 s_t).
The network (1216 -> 256 GELU -> 256 GELU -> 12 = mean and log-scale) is
trained with the Gaussian negative log-likelihood and Adam, all on the GPU
with the library's BF16 matrix-core kernels.

Usage: python -m paper_2105_05600_amd.train_proposal --sequences 192 --epochs 150 \
           --kappas 1.5,2,3,4 --deltas 0.005,0.01,0.02 --eval-sequences 6 --eval-frames 120
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
import synth.mlp_init as mlp_init  # noqa: E402
from paper_2105_05600_amd import rose  # noqa: E402

FEATURE_DIM = 1216
LOW_W, LOW_H = 40, 30


def log(msg):
    print(f"[train] {msg}", flush=True)


def make_sequence(seed: int, n_frames: int, width: int, height: int, speed=None):
    rng = np.random.default_rng(seed)
    v = float(rng.uniform(1.0, 4.0)) if speed is None else speed
    return synth.room_sequence(scene_seed=seed, traj_seed=seed + 1, noise_seed=seed + 2, n_frames=n_frames,
                               speed=v, ang_speed=0.67 * v, width=width, height=height)


def low_camera(K, scale):
    return synth.Intrinsics(LOW_W, LOW_H, K.fx / scale, K.fy / scale, (K.cx + 0.5) / scale - 0.5,
                            (K.cy + 0.5) / scale - 0.5)


def features(vol, depth, K, scale, q, t, vel):
    render = rose.raycast(vol, q, t, low_camera(K, scale), near=0.2, far=8.0, step=0.005)
    return rose.proposal_features(depth, K, render, low_camera(K, scale), scale, vel, FEATURE_DIM)


def generate(seeds, n_frames, width, height, chunk, workers, gpu_render=False):
    """Plain-PST pairs (X, Y) from the sequences `seeds` (GPU).  gpu_render:
    the depth frames are rendered on the GPU (synth.gpu_render, seeded torch
    noise) instead of on the host."""
    scale = width // LOW_W
    Xs, Ys = [], []
    pst = rose.pst_sample(10240, 5600)
    for c0 in range(0, len(seeds), chunk):
        group = seeds[c0:c0 + chunk]
        seqs = [make_sequence(s, n_frames, width, height) for s in group]
        t0 = time.perf_counter()
        if gpu_render:
            from synth.gpu_render import render_depths
            depths = [list(render_depths(sq.scene, sq.K, sq.poses[:n_frames], sq.zmin, sq.zmax,
                                         noise_seed=sq.noise_seed, noise_k=sq.noise_k, device="cuda"))
                      for sq in seqs]
        else:
            depths = [[torch.from_numpy(d).cuda() for d in sq.depths(range(n_frames), workers=workers)]
                      for sq in seqs]
        log(f"sequences {c0}..{c0 + len(group) - 1}: rendered in {time.perf_counter() - t0:.1f} s")
        vols = [rose.Tsdf(sq.dims, sq.vox, sq.mu, sq.origin) for sq in seqs]
        params = [rose.track_params(max_iters=20, stride=4) for _ in seqs]
        batch = rose.Batch(vols, [sq.K for sq in seqs], [pst] * len(seqs), params)
        states = (rose.TrackState * len(seqs))(*[rose.track_state(sq.poses[0].q, sq.poses[0].t, [1.0] * 6,
                                                                  tsdf_built=False) for sq in seqs])
        batch.track([d[0] for d in depths], states)
        for i, sq in enumerate(seqs):
            vols[i].integrate(depths[i][0], sq.K, sq.poses[0].q, sq.poses[0].t)
            states[i].tsdf_built = 1
        prev = [(list(sq.poses[0].q), list(sq.poses[0].t)) for sq in seqs]
        vel = [[0.0] * 6 for _ in seqs]
        t1 = time.perf_counter()
        for f in range(1, n_frames):
            feats = [features(vols[i], depths[i][f], seqs[i].K, scale, prev[i][0], prev[i][1], vel[i])
                     for i in range(len(seqs))]
            res = batch.track([d[f] for d in depths], states)
            for i, sq in enumerate(seqs):
                q, t = res[i]["q"], res[i]["t"]
                u = rose.chart_log(prev[i][0], prev[i][1], q, t)
                if f >= 2 and res[i]["status"] == 0:
                    Xs.append(feats[i])
                    Ys.append(torch.tensor(u, dtype=torch.float32))
                vel[i] = u
                prev[i] = (q, t)
                vols[i].integrate(depths[i][f], sq.K, q, t)
        torch.cuda.synchronize()
        log(f"  tracked {len(seqs)} x {n_frames - 1} frames in {time.perf_counter() - t1:.1f} s; pairs {len(Xs)}")
        batch.close()
        for v in vols:
            v.close()
        del vols, depths
        torch.cuda.empty_cache()
    X = torch.stack(Xs).cuda().contiguous()
    Y = torch.stack(Ys).cuda().contiguous()
    return X, Y


def train(X, Y, epochs, batch, lr, seed):
    """Adam on the Gaussian NLL with a cosine learning-rate decay to lr/20."""
    net = rose.Mlp(FEATURE_DIM, 256, 12, max_batch=batch)
    P = net.pack(mlp_init.init_params(seed))
    G = torch.zeros_like(P)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    n = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    step = 0
    hist = []
    steps_total = max(1, epochs * (n // batch))
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).cuda()
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb = X[idx].contiguous()
            yb = Y[idx].contiguous()
            net.loss_grad(P, xb, yb, G, loss)
            step += 1
            lr_t = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * min(step, steps_total) / steps_total)))
            rose.Mlp.adam(P, G, M, V, step, lr_t)
            tot += float(loss.item())
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if ep % 5 == 0 or ep == epochs - 1:
            log(f"epoch {ep}: mean NLL {hist[-1]:.4f}")
    return net, P, hist


def evaluate(net, P, seeds, n_frames, width, height, n_small=4096, workers=16, kappa=2.0, delta=0.01,
             modes=("plain", "learned"), nets=None, learned_iters=0):
    """Plain 10240-particle PST vs learned proposal + 4096 particles with the
    plain fallback, on identical held-out sequences: ATE (RMSE, Horn
    alignment) and frames/s of the tracking calls.  `nets` optionally maps
    further mode names to other parameter vectors (e.g. an untrained
    network) run like "learned"."""
    scale = width // LOW_W
    pst_plain = rose.pst_sample(10240, 5600)
    pst_small = rose.pst_sample(n_small, 5600)
    work = torch.zeros(LOW_W * LOW_H + FEATURE_DIM + 12, dtype=torch.float32, device="cuda")
    lp = rose.learned_params(scale=scale, kappa=kappa, delta=delta, iters=learned_iters)
    nets = dict(nets or {})
    nets.setdefault("learned", P)
    out = []
    for seed in seeds:
        sq = make_sequence(seed, n_frames, width, height)
        depths = [torch.from_numpy(d).cuda() for d in sq.depths(range(n_frames), workers=workers)]
        gt = np.array([p.t for p in sq.poses[:n_frames]])
        row = {"seed": seed}
        for mode in modes:
            vol = rose.Tsdf(sq.dims, sq.vox, sq.mu, sq.origin)
            params = rose.track_params(max_iters=20, stride=4)
            st = rose.track_state(sq.poses[0].q, sq.poses[0].t, [1.0] * 6, tsdf_built=False)
            rose.track_frame(vol, depths[0], sq.K, pst_plain, params, st)
            vol.integrate(depths[0], sq.K, sq.poses[0].q, sq.poses[0].t)
            st.tsdf_built = 1
            est = [np.array(sq.poses[0].t)]
            prev = (list(sq.poses[0].q), list(sq.poses[0].t))
            vel = [0.0] * 6
            fallbacks = 0
            evals = 0.0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for f in range(1, n_frames):
                if mode == "plain":
                    r = rose.track_frame(vol, depths[f], sq.K, pst_plain, params, st)
                    evals += 10240 * sum(r["n_overlap"])
                else:
                    r = rose.track_frame_learned(vol, depths[f], sq.K, pst_small, pst_plain, net, nets[mode], work,
                                                 vel, params, lp, st)
                    fallbacks += int(r["fallback"])
                    # the stats are the final run's (the plain rerun after a fallback)
                    evals += sum(n * o for n, o in zip(r["n_particles"], r["n_overlap"]))
                q, t = list(st.pose.q), list(st.pose.t)
                vel = rose.chart_log(prev[0], prev[1], q, t)
                prev = (q, t)
                est.append(np.array(t))
                vol.integrate(depths[f], sq.K, q, t)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            _, rmse = synth.ate(np.array(est), gt)
            row[mode] = {"ate_rmse_m": rmse, "frames_per_s": (n_frames - 1) / dt, "fallbacks": fallbacks,
                         "evals": evals}
            vol.close()
        log(f"eval seed {seed}: {json.dumps(row)}")
        out.append(row)
    return out


def summarize(rows, modes):
    """Mean ATE and total frames/s per mode over evaluated sequences."""
    res = {}
    for m in modes:
        ate = [r[m]["ate_rmse_m"] for r in rows]
        fps = [r[m]["frames_per_s"] for r in rows]
        res[m] = {"ate_rmse_mean_m": float(np.mean(ate)), "frames_per_s_mean": float(np.mean(fps)),
                  "fallbacks": int(sum(r[m].get("fallbacks", 0) for r in rows))}
    return res


def save(path, net, P, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    parts = net.unpack(P.detach().cpu())
    np.savez(path, **{k: v.numpy() for k, v in parts.items()})
    with open(os.path.splitext(path)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)


def load(path):
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in ("W1", "b1", "W2", "b2", "W3", "b3")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sequences", type=int, default=64)
    ap.add_argument("--frames", type=int, default=160)
    ap.add_argument("--width", type=int, default=320)
    ap.add_argument("--height", type=int, default=240)
    ap.add_argument("--chunk", type=int, default=16)
    ap.add_argument("--gpu-render", action="store_true", help="render the training frames on the GPU")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--load", default=None, help="skip data generation and training; load these weights")
    ap.add_argument("--kappas", default="2", help="comma-separated kappa values tried on the validation set")
    ap.add_argument("--deltas", default="0.01", help="comma-separated fallback deltas tried on the validation set")
    ap.add_argument("--variants", default="4096:20",
                    help="comma-separated particles:iterations of the learned run tried on the validation set")
    ap.add_argument("--val-sequences", type=int, default=4)
    ap.add_argument("--val-frames", type=int, default=60)
    ap.add_argument("--eval-sequences", type=int, default=4)
    ap.add_argument("--eval-frames", type=int, default=90)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                                                  "proposal.npz"))
    args = ap.parse_args()
    torch.cuda.set_device(0)
    meta = {}
    if args.load:
        net = rose.Mlp(FEATURE_DIM, 256, 12, max_batch=args.batch)
        P = net.pack(load(args.load))
        with open(os.path.splitext(args.load)[0] + ".json") as f:
            meta = json.load(f)
        meta.pop("eval", None)
        meta.pop("validation", None)
    else:
        seeds = [10000 + 10 * i for i in range(args.sequences)]
        t0 = time.perf_counter()
        X, Y = generate(seeds, args.frames, args.width, args.height, args.chunk, args.workers, args.gpu_render)
        t_gen = time.perf_counter() - t0
        log(f"{X.shape[0]} pairs in {t_gen:.1f} s; |y| mean {Y.abs().mean(0).tolist()}")
        t0 = time.perf_counter()
        net, P, hist = train(X, Y, args.epochs, args.batch, args.lr, seed=1)
        t_train = time.perf_counter() - t0
        meta = {"pairs": int(X.shape[0]), "sequences": args.sequences, "frames": args.frames,
                "image": [args.width, args.height], "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
                "generation_s": t_gen, "training_s": t_train, "nll_history": hist}
        del X, Y
    # learned-run settings chosen on validation sequences (seeds 30000+), never
    # on the test sequences: the fastest setting whose mean ATE is at most
    # plain PST's, else the one with the lowest mean ATE
    val_seeds = [30000 + 10 * i for i in range(args.val_sequences)]
    plain_val = summarize(evaluate(net, P, val_seeds, args.val_frames, args.width, args.height,
                                   workers=args.workers, modes=("plain",)), ("plain",))["plain"]
    log(f"validation plain: {json.dumps(plain_val)}")
    variants = [tuple(int(x) for x in v.split(":")) for v in args.variants.split(",")]
    grid = [(float(k), float(d), n, it) for k in args.kappas.split(",") for d in args.deltas.split(",")
            for n, it in variants]
    val = []
    for kappa, delta, n_small, iters in grid:
        rows = evaluate(net, P, val_seeds, args.val_frames, args.width, args.height, n_small=n_small,
                        workers=args.workers, kappa=kappa, delta=delta, modes=("learned",), learned_iters=iters)
        sm = summarize(rows, ("learned",))["learned"]
        val.append({"kappa": kappa, "delta": delta, "particles": n_small, "iters": iters, **sm})
        log(f"validation kappa {kappa} delta {delta} particles {n_small} iters {iters}: {json.dumps(sm)}")
    ok = [v for v in val if v["ate_rmse_mean_m"] <= plain_val["ate_rmse_mean_m"]]
    best = max(ok, key=lambda v: v["frames_per_s_mean"]) if ok else min(val, key=lambda v: v["ate_rmse_mean_m"])
    log(f"chosen: {json.dumps(best)}")
    untrained = net.pack(mlp_init.init_params(1))
    ev = evaluate(net, P, [20000 + 10 * i for i in range(args.eval_sequences)], args.eval_frames, args.width,
                  args.height, n_small=best["particles"], workers=args.workers, kappa=best["kappa"],
                  delta=best["delta"], modes=("plain", "learned", "untrained"), nets={"untrained": untrained},
                  learned_iters=best["iters"])
    meta.update({"kappa": best["kappa"], "delta": best["delta"], "particles": best["particles"],
                 "iters": best["iters"], "validation_plain": plain_val, "validation": val, "eval": ev,
                 "eval_summary": summarize(ev, ("plain", "learned", "untrained"))})
    log(f"test summary: {json.dumps(meta['eval_summary'])}")
    save(args.out, net, P, meta)
    log(f"saved {args.out}")


if __name__ == "__main__":
    main()
