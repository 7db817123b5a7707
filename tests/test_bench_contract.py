"""bench.py contract checks that need no GPU: more than one GPU is refused
with a message before any device work, and the traffic figure is taken
and issued-instruction figures are taken from the committed counter summary
only while it matches the kernel source."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_figures_match_current_source_or_are_absent():
    import bench
    from paper_2007_10752_amd import costs
    pmc = bench.pmc_from_profile("bitslice", 1 << 30)
    with open(os.path.join(ROOT, "profiles", "bitslice_1gib_pmc.md")) as f:
        text = f.read()
    current = bench.kernel_source_hash("bitslice")
    if "source_sha256=%s" % current in text:
        t = pmc["bytes_per_launch"]
        assert 2 * (1 << 30) <= t < 1.01 * 2 * (1 << 30)
        # issued VALU lane operations at least the algorithmic count, and
        # not far above it
        issued = pmc["valu_insts_per_launch"] * 64
        algo = costs.ops_per_block("bitslice") * (1 << 27)
        assert algo <= issued < 1.1 * algo
    else:
        assert pmc == {}
    assert bench.pmc_from_profile("bitslice", 1 << 20) == {}  # other workloads: no figure
