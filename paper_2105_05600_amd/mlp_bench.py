"""Throughput of the proposal network's matrix-core kernels (k_gemm_bf16 and
the elementwise kernels around it) at the sizes the learned proposal uses:
one inference per sequence (B = 1, and 32 for a batched frame step), a
training step of B = 1024 samples (forward, NLL loss and gradients, Adam),
and one large GEMM (4096^3) for the kernel itself away from the latency of
small shapes.  Times from HIP events on the launch stream over repeated
calls; work counted as the GEMMs' 2 M N K flops: forward 2 B (in h + h h +
h o), a training step twice the forward plus the input gradients of the
second and third layers, 2 B (h h + h o).  Peak: MI355X dense BF16, 2.5
PFLOP/s.

    python -m paper_2105_05600_amd.mlp_bench                      # one JSON line
    python -m paper_2105_05600_amd.mlp_bench --summary TRACE_DIR --bench-json FILE --out FILE --command CMD

The second form writes a markdown summary of a `rocprofv3 --kernel-trace
--stats` run of the first beside its JSON line."""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys

import numpy as np
import torch

PEAK_BF16_FLOPS = 2.5e15
IN, HID, OUT = 1216, 256, 12


def _time(fn, reps: int, warm: int = 3) -> float:
    """Average milliseconds of fn() over reps calls (HIP events on the
    current stream, which the library's calls use)."""
    for _ in range(warm):
        fn()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def run() -> dict:
    from paper_2105_05600_amd import rose
    import synth.mlp_init as mlp_init
    torch.cuda.set_device(0)
    g = torch.Generator(device="cpu").manual_seed(7)
    net = rose.Mlp(IN, HID, OUT, max_batch=1024)
    P = net.pack(mlp_init.init_params(3))
    fwd_flops = 2.0 * (IN * HID + HID * HID + HID * OUT)
    out = {"metric": "proposal network on the matrix cores: TFLOP/s of forward passes, training steps and one "
                     "large GEMM", "peak_tflops": PEAK_BF16_FLOPS / 1e12, "dtype": "bf16 operands, f32 accumulation"}
    for B in (1, 32, 1024):
        X = torch.randn(B, IN, generator=g).cuda()
        ms = _time(lambda: net.forward(P, X), reps=200 if B < 1024 else 100)
        tf = fwd_flops * B / (ms * 1e-3) / 1e12
        out[f"forward_B{B}"] = {"ms": ms, "tflops": tf, "frac": tf * 1e12 / PEAK_BF16_FLOPS}
    B = 1024
    X = torch.randn(B, IN, generator=g).cuda()
    Y = (torch.randn(B, 6, generator=g) * 0.05).cuda()
    grads = torch.zeros_like(P)
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    loss = torch.zeros(1, device="cuda")
    step = [0]

    def train_step():
        step[0] += 1
        net.loss_grad(P, X, Y, grads, loss)
        rose.Mlp.adam(P, grads, m, v, step[0], 1e-4)

    ms = _time(train_step, reps=100)
    tr_flops = 2.0 * fwd_flops * B + 2.0 * B * (HID * HID + HID * OUT)
    tf = tr_flops / (ms * 1e-3) / 1e12
    out[f"train_step_B{B}"] = {"ms": ms, "tflops": tf, "frac": tf * 1e12 / PEAK_BF16_FLOPS}
    n = 4096
    A = torch.randn(n, n, generator=g).cuda()
    Bm = torch.randn(n, n, generator=g).cuda()
    ms = _time(lambda: rose.gemm_bf16(A, Bm), reps=20)
    tf = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
    out["gemm_4096"] = {"ms": ms, "tflops": tf, "frac": tf * 1e12 / PEAK_BF16_FLOPS}
    net.close()
    return out


def summary(trace_dir: str, bench_json: str, command: str) -> str:
    rows = []
    for fn in glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True):
        with open(fn, newline="") as f:
            rows += list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    with open(bench_json) as f:
        bench = json.loads(f.read().strip().splitlines()[-1])
    lines = ["# k_gemm_bf16 and the proposal network's kernels (forward, training step, 4096^3 GEMM)", "",
             "rocprofv3 kernel-trace statistics of one mlp_bench.py run (MI355X, gfx950).", "",
             "Command (repository root, after `cd /tmp && export TMPDIR=/tmp` and back):", "", f"    {command}", "",
             "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows[:12]:
        name = r["Name"] if len(r["Name"]) <= 90 else r["Name"][:87] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    lines += ["", "The run's own timing (HIP events; TFLOP/s of the GEMM work, fraction of the 2.5 PFLOP/s dense "
              "BF16 peak):", ""]
    for k, v in bench.items():
        if isinstance(v, dict) and "tflops" in v:
            lines.append(f"* {k}: {v['ms']:.4f} ms, {v['tflops']:.2f} TFLOP/s, frac {v['frac']:.4f}")
    return "\n".join(lines) + "\n"


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--summary", default=None, metavar="TRACE_DIR")
    ap.add_argument("--bench-json", default=None)
    ap.add_argument("--out", default=None)
    ap.add_argument("--command", default="")
    a = ap.parse_args(argv)
    if a.summary:
        md = summary(a.summary, a.bench_json, a.command)
        with open(a.out, "w") as f:
            f.write(md)
        print(md)
        return 0
    print(json.dumps(run()), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
