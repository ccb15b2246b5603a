"""Host-only check of the pass programs (CPU): builds and runs csrc/schedule_check.cpp.

The library launches the line-pass sequences produced by msl_passes.hpp; this
test executes exactly those descriptors with an FP64 line engine on the CPU
and compares with direct 2-D evaluations (forward, checkpoints, far field,
far-field adjoint, checkpointed adjoint), for both propagators.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2212_01253_amd", "csrc", "schedule_check.cpp")


def test_pass_programs_compose(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "schedule_check")
    subprocess.run([hipcc, "--offload-host-only", "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"),
                    "-o", exe, SRC], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("OK")
