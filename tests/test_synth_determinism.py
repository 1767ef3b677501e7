"""The synthetic inputs are bit-reproducible: the same room frames rendered
by two fresh processes, each with 8 render threads, are identical bytes.
(The renderer once rotated its rays with a BLAS product, whose rounding
could change with the library's threading, so that frames differed between
runs.)"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = ("import hashlib, synth; s = synth.room_sequence(); d = s.depths(range(6), workers=8); "
        "print(hashlib.sha256(b''.join(x.tobytes() for x in d)).hexdigest())")


def test_room_frames_identical_across_processes():
    env = dict(os.environ, PYTHONPATH=ROOT)
    outs = [subprocess.run([sys.executable, "-c", CODE], cwd=ROOT, env=env, capture_output=True, text=True,
                           check=True, timeout=300).stdout.strip() for _ in range(2)]
    assert len(outs[0]) == 64 and outs[0] == outs[1]
