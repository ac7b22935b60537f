"""The algorithmic flop count per photon-step used by the benchmark's roofline
is the count produced by instantiating the kernel's own step template with a
counting number type (csrc/flopcount.cpp)."""
import json
import os
import subprocess

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_flop_count_matches_benchmark_constant(tmp_path):
    src = os.path.join(ROOT, "paper_1303_5057_amd", "csrc", "flopcount.cpp")
    exe = str(tmp_path / "flopcount")
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O1", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.dirname(src), src, "-o", exe], check=True, capture_output=True)
    out = json.loads(subprocess.run([exe], check=True, capture_output=True, text=True).stdout)
    assert out["flags"] == 0
    assert out["step_flops"] == bench.F_STEP["fp64"]
    assert 80 < out["rhs_flops"] < out["step_flops"] / 4
