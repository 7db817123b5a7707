"""Search for the S-box gate networks and store them in sbox_networks.txt.

Builds sbox_synth.cpp with g++, runs it once per S-box (restarts split over
worker processes with distinct seeds) and keeps the smallest network found.
Run by hand when the search changes; the committed sbox_networks.txt is what
the emitter reads, so a normal build does not search.

    python -m paper_2007_10752_amd.gen.synth_sboxes --restarts 2000 --jobs 8
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import tempfile

from .des_tables import SBOX
from .networks import NETWORKS_PATH, format_networks, load_networks, parse_network, verify_network

HERE = os.path.dirname(os.path.abspath(__file__))


def _build(tmpdir):
    exe = os.path.join(tmpdir, "sbox_synth")
    subprocess.run(["g++", "-O2", "-o", exe, os.path.join(HERE, "sbox_synth.cpp")], check=True)
    return exe


def _run(exe, box, restarts, seed):
    vals = [str(v) for row in SBOX[box] for v in row]
    r = subprocess.run([exe, str(restarts), str(seed)] + vals, check=True,
                       capture_output=True, text=True)
    return parse_network(r.stdout)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--restarts", type=int, default=1000)
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 4)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--boxes", default="0,1,2,3,4,5,6,7")
    args = ap.parse_args()
    boxes = [int(b) for b in args.boxes.split(",")]
    try:
        best = load_networks()
    except FileNotFoundError:
        best = {}
    with tempfile.TemporaryDirectory() as td:
        exe = _build(td)
        per_job = max(1, args.restarts // args.jobs)
        with cf.ThreadPoolExecutor(args.jobs) as pool:
            futs = {}
            for box in boxes:
                for j in range(args.jobs):
                    seed = args.seed * 1000003 + box * 7919 + j
                    futs[pool.submit(_run, exe, box, per_job, seed)] = box
            for fut in cf.as_completed(futs):
                box = futs[fut]
                net = fut.result()
                verify_network(box, net)
                if box not in best or len(net["gates"]) < len(best[box]["gates"]):
                    best[box] = net
    for box in sorted(best):
        print("S%d: %d gates" % (box + 1, len(best[box]["gates"])))
    with open(NETWORKS_PATH, "w") as f:
        f.write(format_networks(best))


if __name__ == "__main__":
    main()
