"""Host check of the staging ring that carries per-launch arguments to the
device without synchronising: compiled with g++ and run against a simulated
in-order stream (no GPU)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_staging_ring_never_overwrites_live_regions(tmp_path):
    exe = tmp_path / "ring_check"
    src = os.path.join(ROOT, "tests", "staging_ring_check.cpp")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-o", str(exe), src], check=True)
    out = subprocess.run([str(exe), "100000"], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "errors 0" in out.stdout
