"""Summarise rocprofv3 output of the benchmark into the counter summary that
bench.py reads (HBM traffic, L1 -> L2 read bytes, VALU work and stalls of
the fitness kernel per fitness step).

Usage (repository root), after a kernel-trace run and the counter passes of
the same bench.py command, each pass in its own rocprofv3 run:

    python -m paper_2105_05600_amd.counters --trace DIR --pmc DIR [DIR ...] \
        --bench-json FILE --copy-mib 1024 --steps 20 --warmup 5 --out FILE

--trace: a `rocprofv3 --kernel-trace` output directory; --pmc: one
`rocprofv3 --pmc ...` output directory per pass; --bench-json: the JSON line
bench.py printed in the kernel-trace run (evaluations per fitness step);
--copy-mib: the size of bench.py's --copy-probe, whose FETCH_SIZE and
WRITE_SIZE readings scale those counters to bytes.  --stats-out FILE also
writes the kernel-trace statistics (per kernel: calls, average, min, max,
share of GPU time) with bench.py's own timing of the same run beside them.

A fitness step is one iteration's fitness launches (two in the switching
mode: both kernels are launched, the one whose regime does not hold exits at
once); the timed window is the last steps x iterations steps of the run.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("fitness.hip", "common.h")]
VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock (non-packed issue)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def is_fitness(name: str) -> bool:
    """The fitness kernel's instances (not its reduce, finish or batch
    kernels), with or without the namespace in the demangled name."""
    return re.search(r"(^|[\s:])k_fitness<", name) is not None


def _rows(pattern: str):
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise SystemExit(f"no file matches {pattern}")
    for fn in files:
        with open(fn, newline="") as f:
            yield from csv.DictReader(f)


def trace_steps(trace_dir: str, n_steps: int):
    """Durations (ns) of the last n_steps fitness steps, and the kernel names
    of a step."""
    rows = [r for r in _rows(os.path.join(trace_dir, "**", "*kernel_trace.csv")) if is_fitness(r["Kernel_Name"])]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    names = sorted({r["Kernel_Name"] for r in rows[-2 * n_steps:]})
    per = len(names) if len(names) in (1, 2) else 1
    rows = rows[-per * n_steps:]
    dur = np.array([int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows], float)
    return dur.reshape(n_steps, per).sum(axis=1), names


def _shape_of(name: str) -> str:
    """'P,U' of a k_fitness instance name (its first two template arguments)."""
    m = re.search(r"k_fitness<\s*(\d+),\s*(\d+)", name)
    return f"{m.group(1)},{m.group(2)}" if m else name


def pmc_steps(pmc_dir: str, n_steps: int, per: int):
    """Per counter: its value summed over the dispatches of each of the last
    n_steps fitness steps; per counter and kernel shape ('P,U'), its total
    over those dispatches; and the copy probe's readings."""
    vals = {}
    names = {}
    copy = {}
    for r in _rows(os.path.join(pmc_dir, "**", "*counter_collection.csv")):
        name, c, v, d = r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"]), int(r["Dispatch_Id"])
        if is_fitness(name):
            vals.setdefault(c, {}).setdefault(d, 0.0)
            vals[c][d] += v
            names[d] = _shape_of(name)
        elif "vectorized_elementwise_kernel" in name and ("AUnaryFunctor" in name or "MulFunctor" in name):
            copy.setdefault(c, []).append(v)  # the copy probe's multiply by one
    out, by_shape = {}, {}
    for c, byd in vals.items():
        ds = sorted(byd)[-per * n_steps:]
        out[c] = np.array([byd[d] for d in ds]).reshape(n_steps, per).sum(axis=1)
        for d in ds:
            by_shape.setdefault(c, {}).setdefault(names[d], 0.0)
            by_shape[c][names[d]] += byd[d]
    return out, by_shape, copy


def kernel_stats_md(trace_dir: str, bench: dict, dur_ns, names, command: str) -> str:
    """Markdown summary of a `rocprofv3 --kernel-trace --stats` run."""
    rows = list(_rows(os.path.join(trace_dir, "**", "*kernel_stats.csv")))
    rf = bench["roofline"]
    lines = ["# k_fitness on the 512^3 room sequence (640x480 stride 4, 10240 particles, 20 iterations)", "",
             "rocprofv3 kernel-trace statistics of the default bench.py run (MI355X, gfx950, 256 CUs).", ""]
    if command:
        lines += ["Command (repository root, after `cd /tmp && export TMPDIR=/tmp` and back; `--no-cpu-baseline`",
                  "only skips the host-side oracle timing):", "", "    " + command, ""]
    lines += [f"Kernels of a fitness step: {', '.join('`' + n + '`' for n in names)}.", "",
              "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"] if len(r["Name"]) <= 90 else r["Name"][:87] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    ms = float(rf["avg_launch_ms"])
    lines += ["", f"bench.py's HIP-event average per fitness step in the same run: {ms * 1e3:.1f} us; rocprofv3, "
              f"the sum of the step's kernel durations over the same window: {dur_ns.mean() / 1e3:.1f} us.",
              f"Algorithmic bytes per step: {rf['bytes_per_eval']:.0f} B x {rf['evals_per_launch']:.4g} "
              f"particle-point evaluations = {rf['bytes_per_eval'] * rf['evals_per_launch'] / 1e6:.0f} MB -> "
              f"{rf['achieved']:.0f} GB/s; measured L2 -> CU read peak {rf['peak']:.0f} GB/s (frac "
              f"{rf['frac']:.3f}); vs the 8 TB/s HBM peak {rf['hbm']['frac']:.3f}.",
              f"Bench line of this run: {bench['value']:.4g} {bench['unit']}, "
              f"{bench['frames_per_s']:.1f} frames/s, fitness kernel "
              f"{bench['fitness_kernel_evals_per_s']:.4g} evals/s."]
    return "\n".join(lines) + "\n"


def batch_stats_md(trace_dir: str, bench_json: str, command: str) -> str:
    """Markdown summary of a kernel-trace run of bench_batch.py: per kernel
    calls, average, min, max and share of GPU time, with the run's own
    frames/s of both paths."""
    rows = list(_rows(os.path.join(trace_dir, "**", "*kernel_stats.csv")))
    with open(bench_json) as f:
        b = json.loads([ln for ln in f if ln.startswith("{")][-1])
    lines = [f"# Batched tracking of {b['sequences']} uneven sequences ({b['frames']} frames each)", "",
             "rocprofv3 kernel-trace statistics of one bench_batch.py run (MI355X, gfx950): the launch-shape",
             "tuning, the batched run and the same sequences one after another through the single path.", ""]
    if command:
        lines += ["Command (repository root, after `cd /tmp && export TMPDIR=/tmp` and back):", "",
                  "    " + command, ""]
    lines += ["| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows[:24]:
        name = r["Name"] if len(r["Name"]) <= 90 else r["Name"][:87] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    lines += ["", f"Run: batch shape {b['shape']} (tuning, ms per frame step: {b['tune_ms_per_step']}); "
              f"batched {b['batch']['frames_per_s']:.1f} frames/s ({b['batch']['evals_per_s']:.3e} evals/s), "
              f"one after another {b['single']['frames_per_s']:.1f} frames/s; speed-up {b['speedup']:.3f}; "
              f"poses identical: {b['poses_identical']}; mean ATE {b['ate_rmse_m']['mean']:.4f} m."]
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--pmc", nargs="*", default=[])
    ap.add_argument("--bench-json", required=True)
    ap.add_argument("--batch", action="store_true",
                    help="the trace is of bench_batch.py: write only its kernel statistics to --out")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--command", default="")
    ap.add_argument("--out", required=True)
    ap.add_argument("--stats-out", default=None)
    ap.add_argument("--stats-command", default="")
    a = ap.parse_args(argv)
    if a.batch:
        md = batch_stats_md(a.trace, a.bench_json, a.command)
        with open(a.out, "w") as f:
            f.write(md)
        print(md)
        return 0
    n_steps = a.steps * a.iters
    with open(a.bench_json) as f:
        bench = json.loads([ln for ln in f if ln.startswith("{")][-1])
    evals = float(bench["roofline"]["evals_per_launch"])
    dur, names = trace_steps(a.trace, n_steps)
    per = len(names)
    counters, by_shape, copy = {}, {}, {}
    for d in a.pmc:
        c, bs, cp = pmc_steps(d, n_steps, per)
        counters.update(c)
        by_shape.update(bs)
        for k, v in cp.items():
            copy.setdefault(k, []).extend(v)
    copy_kib = a.copy_mib * 1024.0

    def scale(counter):
        # the copy probe's multiply reads and writes copy_kib KiB per dispatch
        vals = copy.get(counter, [])
        ref = float(np.median(vals)) if vals else 0.0
        return copy_kib / ref if ref > 0 else None

    lines = [f"# k_fitness on the 512^3 room sequence: counters per fitness step", ""]
    lines.append("rocprofv3 counter passes over one bench.py command, one run per pass; the timed window is the")
    lines.append(f"last {n_steps} fitness steps ({a.steps} timed frames x {a.iters} iterations after {a.warmup} warmup "
                 "frames).")
    if a.command:
        lines += ["", "Command (repository root, after `cd /tmp && export TMPDIR=/tmp` and back):", "",
                  "    " + a.command]
    lines += ["", f"Kernels of a fitness step: {', '.join('`' + n + '`' for n in names)}", "",
              "| counter (per fitness step) | mean | min | max |", "|---|---|---|---|"]
    for c in sorted(counters):
        v = counters[c]
        lines.append(f"| {c} | {v.mean():.4g} | {v.min():.4g} | {v.max():.4g} |")
    ms = dur.mean() * 1e-6
    lines += ["", f"Fitness step duration (kernel trace, sum over the step's launches): mean {dur.mean() / 1e3:.1f} us, "
              f"p10 {np.percentile(dur, 10) / 1e3:.1f}, median {np.median(dur) / 1e3:.1f}, "
              f"p90 {np.percentile(dur, 90) / 1e3:.1f} us; evaluations per step {evals:.4g} "
              f"(bench.py, same window)."]
    kv = {"kernel_source_sha256_16": kernel_source_hash(), "lookup": bench["config"].get("lookup", "nearest"),
          "shape": "x".join(str(v) for v in bench["roofline"]["shape"]), "window": f"{a.warmup}+{a.steps}",
          "evals_per_launch": f"{evals:.6g}", "trace_ms_per_launch": f"{ms:.6g}"}
    derived = []
    if "FETCH_SIZE" in counters and "WRITE_SIZE" in counters:
        fs, ws = scale("FETCH_SIZE"), scale("WRITE_SIZE")
        if fs and ws:
            rd = counters["FETCH_SIZE"].mean() * 1024.0 * fs
            wr = counters["WRITE_SIZE"].mean() * 1024.0 * ws
            kv["traffic_bytes_per_launch"] = f"{rd + wr:.6g}"
            derived.append(f"HBM read {rd / 1e6:.1f} MB + write {wr / 1e6:.2f} MB per step (FETCH_SIZE x {fs:.3f}, "
                           f"WRITE_SIZE x {ws:.3f} from the copy probe), {(rd + wr) / (4 * evals):.2f}x the "
                           f"algorithmic 4 B per evaluation; {(rd + wr) / (ms * 1e-3) / 1e12:.2f} TB/s")
    if "TCP_TCC_READ_REQ_sum" in counters:
        req = counters["TCP_TCC_READ_REQ_sum"].mean()
        kv["l2_read_bytes_per_launch"] = f"{req * 128.0:.6g}"
        kv["l2_requests_per_eval"] = f"{req / evals:.4g}"
        derived.append(f"L1 -> L2 read requests {req / evals:.3f} per evaluation; x 128 B = "
                       f"{req * 128 / (ms * 1e-3) / 1e12:.2f} TB/s")
    if "TCP_TOTAL_CACHE_ACCESSES_sum" in counters:
        acc = counters["TCP_TOTAL_CACHE_ACCESSES_sum"].mean()
        kv["l1_accesses_per_eval"] = f"{acc / evals:.4g}"
        if "TCP_TCC_READ_REQ_sum" in counters:
            derived.append(f"L1 accesses {acc / evals:.3f} per evaluation, hit rate "
                           f"{1 - counters['TCP_TCC_READ_REQ_sum'].mean() / acc:.3f}")
    if "TCC_HIT_sum" in counters and "TCC_MISS_sum" in counters:
        h, m = counters["TCC_HIT_sum"].mean(), counters["TCC_MISS_sum"].mean()
        derived.append(f"L2 hit rate {h / (h + m):.3f}")
    if "SQ_INSTS_VALU" in counters:
        ops = counters["SQ_INSTS_VALU"].mean() * 64.0 / evals
        kv["valu_lane_ops_per_eval"] = f"{ops:.4g}"
        derived.append(f"VALU lane-ops per evaluation {ops:.2f} (SQ_INSTS_VALU x 64); the VALU ceiling "
                       f"R_valu = {VALU_LANE_OPS_PER_S:.3e} / {ops:.2f} = {VALU_LANE_OPS_PER_S / ops:.3e} evals/s")
    if "SQ_INSTS_VMEM_RD" in counters:
        derived.append(f"vector memory reads per evaluation {counters['SQ_INSTS_VMEM_RD'].mean() * 64 / evals:.3f}")
    if "TA_ADDR_STALLED_BY_TC_CYCLES_sum" in counters and "TA_BUSY_sum" in counters:
        f = counters["TA_ADDR_STALLED_BY_TC_CYCLES_sum"].mean() / counters["TA_BUSY_sum"].mean()
        kv["ta_stalled_by_tc_frac"] = f"{f:.4g}"
        derived.append(f"the address unit waits on the L1 for {100 * f:.0f}% of its busy cycles")
    if "SQ_INSTS_VALU" in counters:
        # a wave64 VALU instruction holds a 16-lane SIMD for 4 clocks; 1024
        # SIMDs; the clock from GRBM_GUI_ACTIVE (summed over the 8 XCDs) when
        # it was collected, else the nominal 2.4 GHz
        cycles = ms * 1e-3 * 2.4e9
        if "GRBM_GUI_ACTIVE" in counters:
            cycles = counters["GRBM_GUI_ACTIVE"].mean() / 8.0
            derived.append(f"effective clock {cycles / (ms * 1e-3) / 1e9:.2f} GHz (GRBM_GUI_ACTIVE / 8 over the "
                           f"step time)")
        busy = counters["SQ_INSTS_VALU"].mean() * 4.0 / (1024.0 * cycles)
        kv["valu_busy_frac"] = f"{busy:.4g}"
        derived.append(f"VALU busy {100 * busy:.0f}% of the SIMD cycles of a step")
    split = bench["roofline"].get("switch_split")
    if split:
        # per side of the switching mode: totals over the window's dispatches
        # of that kernel (its idle launches included: they exit at once)
        # divided by the evaluations it did (bench.py, same window)
        for side, sd in split.items():
            shp = re.search(r"<(\d+),(\d+)>", sd["kernel"])
            key = f"{shp.group(1)},{shp.group(2)}"
            ev = float(sd["evals"])
            if ev <= 0:
                continue
            parts = [f"{side} ({sd['kernel']}): {sd['steps']} steps, {ev / max(sd['steps'], 1):.4g} evaluations and "
                     f"{sd['ms'] / max(sd['steps'], 1):.3f} ms per step, {sd['evals_per_s']:.3e} evals/s"]
            if key in by_shape.get("SQ_INSTS_VALU", {}):
                ops = by_shape["SQ_INSTS_VALU"][key] * 64.0 / ev
                parts.append(f"VALU lane-ops per evaluation {ops:.2f} (R_valu {VALU_LANE_OPS_PER_S / ops:.3e})")
                kv[f"valu_lane_ops_per_eval_{side}"] = f"{ops:.4g}"
            if key in by_shape.get("TCP_TCC_READ_REQ_sum", {}):
                req = by_shape["TCP_TCC_READ_REQ_sum"][key] / ev
                parts.append(f"L1 -> L2 read requests per evaluation {req:.3f}")
                kv[f"l2_requests_per_eval_{side}"] = f"{req:.4g}"
            if key in by_shape.get("TCP_TOTAL_CACHE_ACCESSES_sum", {}):
                parts.append(f"L1 accesses per evaluation {by_shape['TCP_TOTAL_CACHE_ACCESSES_sum'][key] / ev:.3f}")
            fs = scale("FETCH_SIZE")
            if fs and key in by_shape.get("FETCH_SIZE", {}):
                parts.append(f"HBM read bytes per evaluation {by_shape['FETCH_SIZE'][key] * 1024.0 * fs / ev:.2f}")
            derived.append("; ".join(parts))
    lines += ["", "Derived:"] + [f"* {d}." for d in derived]
    lines += ["", "Values read by bench.py (while the kernel sources hash to the value below and the window and",
              "launch shape match its own):", ""]
    lines += [f"{k}: {v}" for k, v in kv.items()]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    if a.stats_out:
        md = kernel_stats_md(a.trace, bench, dur, names, a.stats_command)
        with open(a.stats_out, "w") as f:
            f.write(md)
        print(md)
    return 0


if __name__ == "__main__":
    sys.exit(main())
