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
    if got:
        assert 6.0e6 < got["traffic_bytes_per_launch"] < 8.0e6 and 5.0 < got["kernel_us_per_launch"] < 20.0
        assert 500 < got["valu_per_wave_row"] < 4000 and 500 < got["valu_per_wave_column"] < 4000
        assert got["waves_per_launch"] == 512
    other = tmp_path / "other.hip"
    other.write_text("// not the kernel source\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", (str(other),))
    assert bench.profile_figures() == {}


def test_roofline_names_the_binding_ceiling():
    # VALU floor 512 waves x 1600 instructions x 64 lanes at 39.3e12/s = 1.33 us is longer
    # than the HBM floor of 6.36 MB at 8 TB/s = 0.79 us: the pass is issue-bound ("alu")
    prof = {"valu_per_wave_row": 1700.0, "valu_per_wave_column": 1500.0, "waves_per_launch": 512,
            "traffic_bytes_per_launch": 6.6e6, "kernel_us_per_launch": 8.0}
    r = bench.roofline(6356992.0, 8e-6, 6.6e6, prof, 512, 512, 6356992.0 / 8e-6 / 1e9, 6.0, 8.0)
    assert r["bound"] == "alu" and r["unit"] == "Tlane-instr/s"
    assert r["valu"]["floor_us"] == pytest.approx(512 * 1600 * 64 / 39.3216e12 * 1e6)
    assert r["frac"] == pytest.approx(r["valu"]["floor_us"] / 8.0)
    assert r["hbm"]["frac"] == pytest.approx(6356992.0 / 8e-6 / 8e12)
    # without the counters the HBM ceiling is the only one reported
    r = bench.roofline(6356992.0, 8e-6, None, {}, 512, 512, 6356992.0 / 8e-6 / 1e9, 6.0, None)
    assert r["bound"] == "hbm" and r["valu"] is None and r["traffic"] is None
