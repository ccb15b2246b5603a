"""Host-side checks of the benchmark's bookkeeping (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_byte_and_flop_models():
    # forward 24 B + checkpoint stores 8/k; recompute 32 B; reverse 40 B
    assert bench.grad_bytes_per_voxel_slice(32) == pytest.approx(96.25)
    assert bench.grad_bytes_per_voxel_slice(1) == pytest.approx(104.0)
    # four 512-point FFTs at 5 n log2 n each, three complex multiplies
    assert bench.fwd_flops_per_voxel_slice(512) == pytest.approx(4 * 5 * 9 + 18)


def test_profile_figures_follow_the_kernel_sources(tmp_path, monkeypatch):
    # the committed summary carries the figures and the hash of the sources it was taken with;
    # any other source text makes the figures unavailable (null in the JSON line)
    got = bench.profile_figures()
    text = open(os.path.join(ROOT, bench.TRAFFIC_PROFILE)).read()
    assert "traffic_bytes_per_launch:" in text and "sources_sha256:" in text
    if got != (None, None):
        b, us = got
        assert 6.0e6 < b < 8.0e6 and 5.0 < us < 20.0
    other = tmp_path / "other.hip"
    other.write_text("// not the kernel source\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", (str(other),))
    assert bench.profile_figures() == (None, None)
