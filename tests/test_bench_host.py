"""Host-side checks of the benchmark's contract (no GPU): more than one GPU
is refused with a message, and the committed rocprofv3 counter summary that
bench.py reads was taken on the current kernel sources, launch shape and
frame window (else the bench line would carry no counter figures)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus_requested"] == 2


def test_counter_summary_matches_the_kernel_sources():
    import bench
    from paper_2105_05600_amd import counters
    assert bench.kernel_source_hash() == counters.kernel_source_hash()
    cnt, why = bench.counter_summary(0, (0, 0), "5+20")
    assert cnt is not None, why
    for k in ("traffic_bytes_per_launch", "l2_read_bytes_per_launch", "l2_requests_per_eval",
              "valu_lane_ops_per_eval", "evals_per_launch", "trace_ms_per_launch"):
        assert cnt.get(k) is not None and cnt[k] > 0, k
