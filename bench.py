"""Benchmark: PST pose search + TSDF fusion on a synthetic fast-motion
sequence, one MI355X.

Workload (one step = one frame): 512^3 TSDF at 1 cm (float psi + float
weight), 640x480 depth (f = 525, noise sigma = 0.002 z^2) stride-4
subsampled, 10240-particle PST, 20 iterations, then fusion of the frame at
the tracked pose.  The camera moves at 3 m/s and 2 rad/s at 30 fps through a
procedural room.  Depth frames are rendered on the host before timing and
are resident in HBM when the timed region starts.

Prints one JSON line: value = particle x point fitness evaluations per
second over the whole timed job (all kernels, all frames); frames/s and ATE
against the synthetic ground truth beside it; the roofline of the fitness
kernel from HIP-event timings; the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# fitness kernel, NEAREST lookup, binary32 TSDF: one 4-byte TSDF gather per
# particle x point evaluation (the paper's per-evaluation data movement)
BYTES_PER_EVAL = {0: 4.0, 1: 32.0}  # binary32 storage; the 16-bit formats move half
FORMATS = {"f32": 0, "f16": 1, "sn16": 2}
HBM_PEAK_GBS = 8000.0
# Sec. 4 multi-resolution PST: (particles, per-axis stride) used in turn; the
# paper does not fix which combination starts a cycle: the densest template
# on the coarsest depth first tracked best on the 6D ablation set
MULTIRES_LEVELS = [(10240, 6), (3072, 4), (1024, 3)]
# measured HBM traffic of the fitness kernel (rocprofv3 FETCH_SIZE + WRITE_SIZE
# on this workload, scaled by the same counters on a copy of known size); it
# is reported only while the kernel sources hash to the value it was taken on
COUNTERS = os.path.join(ROOT, "profiles", "k_fitness_room512_counters.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2105_05600_amd", "csrc", f) for f in ("fitness.hip", "common.h")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--lookup", choices=["nearest", "trilinear"], default="nearest")
    ap.add_argument("--schedule", choices=["single", "multires"], default="single",
                    help="multires: the paper's alternation of (10240, 1/32), (3072, 1/16), (1024, 1/8) as strides "
                         "6, 4, 3")
    ap.add_argument("--fmt", choices=list(FORMATS), default="f32",
                    help="TSDF storage: binary32, binary16 or normalised int16 (arithmetic stays binary32)")
    ap.add_argument("--template", choices=["iid", "poisson"], default="iid",
                    help="poisson: 6D Poisson-disk template (dart throwing, packing fraction 0.03)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--render-workers", type=int, default=16)
    ap.add_argument("--shape", default="0,0", metavar="P,U",
                    help="fitness launch shape (particles per wave, points per lane; 0,0: the switching mode, "
                         "default); 'tune': time every candidate on one frame and keep the fastest")
    ap.add_argument("--switch", default=None, metavar="VOX,DEPTH",
                    help="switching-mode threshold: footprint in voxels, reference depth in metres")
    ap.add_argument("--switch-shape", default=None, metavar="P,U",
                    help="switching mode: the points-across shape used above the threshold (default 4,2)")
    ap.add_argument("--dump-poses", default=None, metavar="FILE",
                    help="write every frame's estimated and true pose (JSON) to FILE")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="before warmup, run a float32 copy of MIB MiB three times (counter calibration)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


L2_NOMINAL_GBS = 39300.0  # 16 channels x 128 B per clock per XCD, 8 XCDs, 2.4 GHz
VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock (one lane-op per lane per clock)


def counter_summary(lookup: int, shape, window: str):
    """The committed counter summary's per-step figures when it was taken on
    the current kernel sources, for this lookup, launch shape and timed
    window; otherwise (None, reason)."""
    try:
        with open(COUNTERS) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith((" ", "|", "*", "#")))
    except OSError:
        return None, "no counter summary"
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None, "counter summary taken on other kernel sources"
    if kv.get("lookup") != ("nearest" if lookup == 0 else "trilinear"):
        return None, "counter summary taken with the other lookup"
    if kv.get("shape") != f"{shape[0]}x{shape[1]}":
        return None, f"counter summary taken with launch shape {kv.get('shape')}"
    if kv.get("window") != window:
        return None, f"counter summary taken over frames {kv.get('window')}, this run {window}"
    out = {}
    for k in ("traffic_bytes_per_launch", "l2_read_bytes_per_launch", "l2_requests_per_eval", "valu_lane_ops_per_eval",
              "ta_stalled_by_tc_frac", "valu_busy_frac", "evals_per_launch", "trace_ms_per_launch"):
        try:
            out[k] = float(kv[k])
        except (KeyError, ValueError):
            out[k] = None
    return out, None


def copy_probe(torch, mib: int):
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"copy probe: 3 x {mib} MiB read + {mib} MiB written")
    del src, dst


def gather_roofline(torch, rose, region_mib: int, reps: int = 5) -> float:
    """4-byte loads per second of the gather-rate probe: every load from its
    own pseudo-random 128-byte line of a region of `region_mib` MiB per XCD
    (2 MiB: L2-resident; 1024 MiB: served by HBM), timed with HIP events on
    the current stream."""
    lines = region_mib * (1 << 20) // 128
    buf = torch.rand(8 * lines * 32, device="cuda")
    blocks, iters = 2048, 64
    sink = torch.zeros(blocks, device="cuda")
    rose.gather_peak(buf, lines, blocks, iters, sink)  # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    loads = 0
    for _ in range(reps):
        loads += rose.gather_peak(buf, lines, blocks, iters, sink)
    e1.record()
    torch.cuda.synchronize()
    del buf, sink
    return loads / (e0.elapsed_time(e1) * 1e-3)


def l2_read_peak(torch, rose, reps: int = 3) -> float:
    """L2 -> CU read bytes per second: coalesced 16-byte loads sweeping a
    2 MiB region per XCD (L2-resident, far larger than a CU's L1), timed
    with HIP events on the current stream."""
    region = 2 * (1 << 20) // 16
    buf = torch.rand(8 * region * 4, device="cuda")
    blocks = 2048
    sink = torch.zeros(blocks, device="cuda")
    rose.l2_read_peak(buf, region, blocks, 1, sink)  # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    nbytes = 0
    for _ in range(reps):
        nbytes += rose.l2_read_peak(buf, region, blocks, 4, sink)
    e1.record()
    torch.cuda.synchronize()
    del buf, sink
    return nbytes / (e0.elapsed_time(e1) * 1e-3)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seq, depth0, depth1, prev_pose, n_particles, lookup):
    """The oracle as it stands (plain C, fitness over particle ranges and
    fusion over z-slices on host threads), timed on this host:
    * frame 1 of the room sequence in full (20 iterations, then fusion) on
      all threads this process may use (at most 16) -> evals/s and frames/s;
    * the first iteration of the same frame on one thread;
    * the small one-frame workload (64^3, 160x120 stride 3, 1024 particles,
      10 iterations) in full, on all threads and on one.
    About 20-40 s of CPU work on a 16-thread host."""
    import oracle
    oracle.build(force=False)
    n_all = max(1, min(16, oracle.host_threads()))
    nx, ny, nz = seq.dims
    psi = np.ones((nz, ny, nx), np.float32)
    wt = np.zeros_like(psi)
    with oracle.threads(n_all):
        oracle.integrate(psi, wt, seq.vox, seq.origin, seq.mu, depth0, seq.K, prev_pose.q, prev_pose.t,
                         prec=oracle.F32)
    pst, _ = oracle.pst_sample(n_particles, 5600)
    args = (psi, seq.vox, seq.origin, depth1, seq.K, pst, prev_pose.q, prev_pose.t, np.full(6, 0.55))
    kw = dict(stride=seq.stride, lookup=lookup, prec=oracle.F32)
    with oracle.threads(n_all):
        t0 = time.perf_counter()
        o = oracle.track_frame(*args, max_iters=seq.iters, **kw)
        t1 = time.perf_counter()
        oracle.integrate(psi, wt, seq.vox, seq.origin, seq.mu, depth1, seq.K, o["q"], o["t"], prec=oracle.F32)
        t2 = time.perf_counter()
    evals = float(n_particles * int(np.sum(o["n_overlap"])))
    with oracle.threads(1):
        t3 = time.perf_counter()
        o1 = oracle.track_frame(*args, max_iters=1, **kw)
        t4 = time.perf_counter()
    evals1 = float(n_particles * int(o1["n_overlap"][0]))
    del psi, wt
    # the small workload in full
    import synth
    w = synth.small_frame()
    sp = np.ones(w.dims[::-1], np.float32)
    sw = np.zeros_like(sp)
    for p, d in zip(w.fuse_poses, w.fuse_depths):
        oracle.integrate(sp, sw, w.vox, w.origin, w.mu, d, w.K, p.q, p.t, prec=oracle.F32)
    spst, _ = oracle.pst_sample(w.n_particles, w.pst_seed)
    prev = w.fuse_poses[-1]
    small = {}
    for n in (n_all, 1):
        with oracle.threads(n):
            ts = time.perf_counter()
            so = oracle.track_frame(sp, w.vox, w.origin, w.depth, w.K, spst, prev.q, prev.t, np.full(6, 0.1),
                                    max_iters=w.iters, stride=w.stride, prec=oracle.F32)
            te = time.perf_counter()
        small[n] = (w.n_particles * int(np.sum(so["n_overlap"])) / (te - ts), te - ts)
    return dict(
        value=evals / (t1 - t0), unit="evals/s", cores=n_all, kind="oracle",
        sample=f"frame 1 of the room sequence in full: {seq.iters} iterations x {n_particles} particles x "
               f"~{o['n_overlap_last']} points on the 512^3 TSDF (whole tracker: overlap, fitness, update), "
               f"{t1 - t0:.1f} s on {n_all} threads; fusion of the frame {t2 - t1:.2f} s",
        frames_per_s=1.0 / (t2 - t0), cpu_model=cpu_model(), nproc=os.cpu_count(),
        threads_available=oracle.host_threads(),
        single_core={"value": evals1 / (t4 - t3), "unit": "evals/s", "cores": 1,
                     "sample": f"iteration 1 of the same frame, {t4 - t3:.1f} s"},
        small_frame={"workload": "64^3 TSDF, 160x120 stride 3, 1024 particles, 10 iterations (whole frame)",
                     "evals_per_s": small[n_all][0], "frames_per_s": 1.0 / small[n_all][1], "cores": n_all,
                     "single_core_evals_per_s": small[1][0], "single_core_frames_per_s": 1.0 / small[1][1]})


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1",
                          "n_gpus_requested": args.gpus}), flush=True)
        sys.exit(2)
    import torch

    import synth
    from paper_2105_05600_amd import rose

    lookup = 0 if args.lookup == "nearest" else 1
    n_frames = 1 + args.warmup + args.steps
    if n_frames > 300:
        raise SystemExit("warmup + steps must be < 300 (sequence length)")
    seq = synth.room_sequence()
    t0 = time.perf_counter()
    depths = seq.depths(range(n_frames), workers=args.render_workers)
    log(f"rendered {n_frames} frames in {time.perf_counter() - t0:.1f} s")
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(torch, args.copy_probe)
    dev_depths = [torch.from_numpy(d).cuda() for d in depths]
    fmt = FORMATS[args.fmt]
    vol = rose.Tsdf(seq.dims, seq.vox, seq.mu, seq.origin, fmt=fmt)
    if args.template == "poisson":
        pst, got, drawn = rose.pst_poisson(seq.n_particles, 5600, rose.poisson_radius(seq.n_particles), 1 << 22)
        if got != seq.n_particles:
            raise SystemExit(f"Poisson-disk template: only {got} rows after {drawn} candidates")
        log(f"Poisson-disk template: {drawn} candidates for {got} rows")
    else:
        pst = rose.pst_sample(seq.n_particles, 5600)
    levels = MULTIRES_LEVELS if args.schedule == "multires" else None
    params = rose.track_params(max_iters=seq.iters, stride=seq.stride, lookup=lookup, levels=levels)
    p0 = seq.poses[0]
    st = rose.track_state(p0.q, p0.t, [1.0] * 6, tsdf_built=False)
    rose.track_frame(vol, dev_depths[0], seq.K, pst, params, st)  # first frame: r_1 = 0.55
    vol.integrate(dev_depths[0], seq.K, p0.q, p0.t)
    st.tsdf_built = 1
    est = [np.array(p0.t)]
    est_q = [np.array(p0.q)]

    def step(i):
        res = rose.track_frame(vol, dev_depths[i], seq.K, pst, params, st)
        vol.integrate(dev_depths[i], seq.K, st.pose.q, st.pose.t)
        est.append(np.array(st.pose.t))
        est_q.append(np.array(st.pose.q))
        return res

    # the launch configuration is set before the warmup frames, so that they
    # run the same kernels as the timed ones
    if args.switch:
        rose.set_fitness_switch(*(float(v) for v in args.switch.split(",")))
    wide = (4, 2)
    if args.switch_shape:
        wide = tuple(int(v) for v in args.switch_shape.split(","))
        rose.set_fitness_switch_shape(*wide)
    if args.shape != "tune":
        shp = tuple(int(v) for v in args.shape.split(","))
        rose.set_fitness_shape(*shp)
        tuned = {"shape": shp, "ms": {}, "cached": False}
    for i in range(1, 1 + args.warmup):
        step(i)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} frames done")
    if args.shape == "tune":
        # launch-shape tuning on the next frame: one tracked frame per
        # compiled shape (from a copy of the state), fitness launches timed
        from paper_2105_05600_amd import autotune
        tuned = autotune.tune_track(vol, dev_depths[1 + args.warmup], seq.K, pst, params, st)
    log(f"fitness shape {tuned['shape']} ({'timed' if args.shape == 'tune' else 'given'}: {tuned['ms']})")
    rose.profile_enable(True)
    rose.profile_reset()
    evals = 0.0
    step_evals, step_mode = [], []  # per timed fitness step: evaluations, kernel that worked
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(1 + args.warmup, n_frames):
        res = step(i)
        evals += float(sum(n * o for n, o in zip(res["n_particles"], res["n_overlap"])))
        step_evals.extend(float(n * o) for n, o in zip(res["n_particles"], res["n_overlap"]))
        step_mode.extend(res["fit_mode"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    prof = rose.profile_read()
    launch_ms = rose.profile_fitness_launches()
    rose.profile_enable(False)
    log(f"timed {args.steps} frames in {wall:.3f} s; profile {prof}")

    gt = np.array([p.t for p in seq.poses[:n_frames]])
    est_a = np.array(est)
    ate_mean, ate_rmse = synth.ate(est_a, gt)
    if args.dump_poses:
        with open(args.dump_poses, "w") as f:
            json.dump({"t_est": est_a.tolist(), "q_est": np.array(est_q).tolist(), "t_true": gt.tolist(),
                       "q_true": [list(map(float, p.q)) for p in seq.poses[:n_frames]],
                       "ate_mean_m": ate_mean, "ate_rmse_m": ate_rmse}, f)
    fit_ms = prof["fitness_ms"] / max(prof["fitness_launches"], 1)
    fit_evals = prof["fitness_evals"] / max(prof["fitness_launches"], 1)
    bytes_per_eval = BYTES_PER_EVAL[lookup] * (1.0 if fmt == 0 else 0.5)
    achieved = fit_evals * bytes_per_eval / (fit_ms * 1e-3) / 1e9
    out = {
        "metric": "particle*point fitness evals/s (+ frames/s at 10k particles; ATE vs ground truth)",
        "value": evals / wall,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"room sequence, 512^3 TSDF @1cm {args.fmt}, 640x480 f=525 stride 4, PST 10240, "
                               "20 iterations + fusion per frame, 3 m/s 2 rad/s",
                   "tsdf": [512, 512, 512], "voxel_m": 0.01, "image": [640, 480], "stride": 4,
                   "particles": seq.n_particles, "iters": seq.iters, "lookup": args.lookup, "schedule": args.schedule,
                   "template": args.template, "tsdf_format": args.fmt},
        "frames_per_s": args.steps / wall,
        "fitness_kernel_evals_per_s": prof["fitness_evals"] / (prof["fitness_ms"] * 1e-3),
        "ate_rmse_m": ate_rmse,
        "ate_mean_m": ate_mean,
        "time_split_ms_per_frame": {"fitness": prof["fitness_ms"] / args.steps,
                                    "update": prof["update_ms"] / args.steps,
                                    "integrate": prof["integrate_ms"] / args.steps},
    }
    shape = tuple(tuned["shape"])
    window = f"{args.warmup}+{args.steps}"
    fit_rate = prof["fitness_evals"] / (prof["fitness_ms"] * 1e-3)
    p_l2 = l2_read_peak(torch, rose)
    g_l2 = gather_roofline(torch, rose, 2)
    g_hbm = gather_roofline(torch, rose, 1024)
    log(f"L2 -> CU reads {p_l2 / 1e12:.2f} TB/s; one-line gathers: L2-resident {g_l2:.3e}/s, "
        f"HBM-resident {g_hbm:.3e}/s; fitness {fit_rate:.3e} evals/s")
    cnt, why = counter_summary(lookup, shape, window) if fmt == 0 else (None, "counters taken for binary32 only")
    elem = 4.0 if fmt == 0 else 2.0
    r_gather = p_l2 / elem  # evaluations/s if every evaluation's element came from L2 at the measured peak
    ops = cnt["valu_lane_ops_per_eval"] if cnt else None
    r_valu = VALU_LANE_OPS_PER_S / ops if ops else None
    if cnt and cnt.get("valu_busy_frac") is not None and cnt["valu_busy_frac"] >= 0.6:
        bound = "alu"
    elif cnt and cnt.get("ta_stalled_by_tc_frac") is not None and cnt["ta_stalled_by_tc_frac"] >= 0.5:
        bound = "l2"
    else:
        bound = "l2"
    achieved_gbs = fit_evals * bytes_per_eval / (fit_ms * 1e-3) / 1e9
    out["roofline"] = {
        "bound": bound,
        "achieved": achieved_gbs, "peak": p_l2 / 1e9, "unit": "GB/s", "frac": achieved_gbs * 1e9 / p_l2,
        "traffic": cnt["traffic_bytes_per_launch"] if cnt else None,
        "what": "fitness step (one iteration's fitness launches) on its gather roofline R_gather = P_L2 / bytes per "
                "TSDF element: achieved = algorithmic bytes (one element per NEAREST evaluation, eight per "
                "TRILINEAR) per step / average step time (HIP events on the launch stream); peak = P_L2, the L2 -> "
                "CU read bandwidth measured in this run (coalesced 16-byte loads, 2 MiB L2-resident region per "
                f"XCD; nominal {L2_NOMINAL_GBS / 1e3:.1f} TB/s); traffic = HBM bytes per step from the committed "
                "rocprofv3 counter summary of the same command and window",
        "kernel": ("k_fitness, switched pair <%d,%d> / <64,8> (one does the work each iteration)" % wide
                   if shape == (0, 0) else f"k_fitness<{shape[0]},{shape[1]}>"),
        "avg_launch_ms": fit_ms, "evals_per_launch": fit_evals, "bytes_per_eval": bytes_per_eval, "shape": list(shape),
        "launch_ms_p10_median_p90": ([float(v) for v in np.percentile(launch_ms, [10, 50, 90])]
                                     if len(launch_ms) else None),
        "window_frames": window, "kernel_source_sha256_16": kernel_source_hash(),
        "hbm": {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS},
        "gather": {"R_gather_evals_per_s": r_gather, "achieved_evals_per_s": fit_rate, "frac": fit_rate / r_gather},
        "valu": ({"lane_ops_per_eval": ops, "R_valu_evals_per_s": r_valu, "frac": fit_rate / r_valu,
                  "busy_frac": cnt.get("valu_busy_frac")} if ops else None),
        "l2_requests_per_eval": cnt["l2_requests_per_eval"] if cnt else None,
        "l1_to_l2_gbs": (cnt["l2_read_bytes_per_launch"] / (fit_ms * 1e-3) / 1e9
                         if cnt and cnt["l2_read_bytes_per_launch"] else None),
        # algorithmic gather bytes over the L1 -> L2 line bytes of the same step
        "coalescing_efficiency": (fit_evals * bytes_per_eval / cnt["l2_read_bytes_per_launch"]
                                  if cnt and cnt["l2_read_bytes_per_launch"] else None),
        "ta_stalled_by_tc_frac": cnt["ta_stalled_by_tc_frac"] if cnt else None,
        "counters": "rocprofv3 summary of the same command and window" if cnt else why,
    }
    if shape == (0, 0) and len(launch_ms) == len(step_mode) and any(step_mode):
        # the switching mode's two sides: steps, evaluations and time of each
        split = {}
        names = {1: "points_across", 2: "particle_per_lane"}
        for mode, name in names.items():
            idx = [j for j, m in enumerate(step_mode) if m == mode]
            ev = sum(step_evals[j] for j in idx)
            ms = float(sum(launch_ms[j] for j in idx))
            wp = (4, 2) if lookup == 1 else wide  # the wide side of trilinear lookups is 4x2
            split[name] = {"kernel": (f"k_fitness<{wp[0]},{wp[1]}>" if mode == 1 else "k_fitness<64,8>"),
                           "steps": len(idx), "evals": ev, "ms": ms,
                           "evals_per_s": ev / (ms * 1e-3) if ms > 0 else None}
        out["roofline"]["switch_split"] = split
    out["gather_probe"] = {
        "what": "not a ceiling: independent 4-byte loads, each from its own pseudo-random 128-byte line of a "
                "region per XCD (2 MiB: L2-resident; 1 GiB: HBM-resident), loads/s",
        "l2_resident_per_s": g_l2, "hbm_resident_per_s": g_hbm, "fitness_evals_per_s": fit_rate}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle: frame 1 in full on all threads, its first iteration on one, the small frame")
        out["cpu_baseline"] = cpu_baseline(seq, depths[0], depths[1], p0, seq.n_particles, lookup)
    print(json.dumps(out), flush=True)
    vol.close()


if __name__ == "__main__":
    main()
