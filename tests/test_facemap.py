"""Host check of the flux work decomposition (csrc/facemap_check.hip): the
same functions the flux kernels use to map blocks and lanes to faces
(direction interleaving, banded cell order, outflow boundary planes) must
take every face of every direction exactly once, for ragged shapes and
every combination of periodic and outflow axes; the reciprocal-based index
splitting must agree with integer division up to 2^32."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1909_01580_amd", "csrc", "facemap_check.hip")


def test_every_face_taken_once(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "facemap_check")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-o", exe, SRC], check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
