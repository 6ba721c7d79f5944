"""The operation counts bench.py uses for the roofline come from the
counting build of the kernels' own per-lane arithmetic; the committed
opcount.json must match what the current sources count."""

import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1909_01580_amd", "csrc", "opcount.hip")
JSON = os.path.join(ROOT, "paper_1909_01580_amd", "opcount.json")


def test_opcount_json_matches_sources(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "opcount")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-o", exe, SRC], check=True, capture_output=True)
    out = json.loads(subprocess.run([exe], check=True, capture_output=True, text=True).stdout)
    assert out == json.load(open(JSON))
    # Sanity: a Gauss-point flux is thousands of operations, dominated by
    # multiplies and adds; a handful of divides and transcendentals.
    assert 1000 < out["flux_gp_ops"] < 20000
    assert out["flux_gp_transcendental"] == 7
