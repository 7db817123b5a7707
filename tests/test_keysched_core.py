"""The lane-parallel key expansion of the batched path (one round key per
lane, computed on its own; mask words formed one round per lane after a
shared walk), checked on the host against the sequential schedule and mask
words of the same header (which the CPU emulation tests pin to the oracle).
Compiled with g++ from tests/keysched_core_check.cpp."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2007_10752_amd", "csrc")


def test_lane_parallel_expansion_equals_sequential(tmp_path):
    exe = str(tmp_path / "keysched_core_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
                    "-o", exe, os.path.join(ROOT, "tests", "keysched_core_check.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
