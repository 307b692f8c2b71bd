"""Host-side behaviour of bench.py, CPU only: it refuses more than one GPU with a
JSON error line, reports a missing GPU the same way, and takes the tile kernel's
HBM traffic from the committed rocprofv3 summary only while that summary was
made from the kernel source as it stands."""
import hashlib
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

KERNELS = os.path.join("paper_1410_5780_amd", "csrc", "pv3d_kernels.hip")
WL = "c3_rooftop_bipv"
PROFILE = os.path.join("profiles", f"tile_{WL}.md")


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_no_gpu_gives_an_error_line():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    r = _run("--steps", "1", "--warmup", "0", "--no-cpu", "--no-extra")
    assert r.returncode == 1
    assert json.loads(r.stdout.strip().splitlines()[-1]) == {"error": "no GPU visible"}


def test_traffic_only_for_the_profiled_kernel_source(tmp_path, monkeypatch):
    for rel in (KERNELS, PROFILE):
        os.makedirs(tmp_path / os.path.dirname(rel), exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), tmp_path / rel)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    src = tmp_path / KERNELS
    prof = tmp_path / PROFILE
    sha = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    text = prof.read_text()
    lines = [ln for ln in text.splitlines() if not ln.startswith("kernel_source_sha256_16 = ")]
    prof.write_text("\n".join(lines + [f"kernel_source_sha256_16 = {sha}", ""]))
    got = bench.measured_traffic("raster", "sparse", WL)
    assert isinstance(got, int) and got > 0
    assert bench.measured_traffic("raster", "materialised", WL) is None
    src.write_bytes(src.read_bytes() + b"\n")          # the kernel changed since the counters were taken
    assert bench.measured_traffic("raster", "sparse", WL) is None
    prof.unlink()
    assert bench.measured_traffic("raster", "sparse", WL) is None


def test_committed_profile_matches_the_kernel_source():
    """The committed rocprofv3 summary was made from the kernels as they stand, so the benchmark's
    traffic figure is a measured one (regenerate the summary after any change to the kernels)."""
    got = bench.measured_traffic("raster", "sparse", WL)
    assert isinstance(got, int) and got > 0


def test_highest_flat_rate_ignores_a_straggler_at_the_lightest_rate():
    import bench
    sweep = [{"rate_hz": 20.0, "p99_ms": 22313.0}, {"rate_hz": 40.0, "p99_ms": 39.7},
             {"rate_hz": 60.0, "p99_ms": 154.8}]
    assert bench.highest_flat_rate(sweep) == 40.0
    assert bench.highest_flat_rate([{"rate_hz": 10.0, "p99_ms": 5.0}, {"rate_hz": 30.0, "p99_ms": 9.9}]) == 30.0
    assert bench.highest_flat_rate([]) is None
