"""bench.py contract checks that need no GPU: more than one GPU is refused
with a message and a non-zero status before anything touches a device."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for n in (2, 8):
        res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                             capture_output=True, text=True, timeout=120, cwd=ROOT)
        assert res.returncode != 0
        assert "one GPU" in res.stderr and f"--gpus {n}" in res.stderr
        assert res.stdout.strip() == ""          # no JSON line
