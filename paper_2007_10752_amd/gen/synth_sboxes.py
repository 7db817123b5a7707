"""Search for the S-box gate networks and store them in sbox_networks.txt.

Builds sbox_synth.cpp with g++, runs it once per S-box and restriction
(restarts split over worker processes with distinct seeds) and keeps, per
box, the network that makes the round cheapest: gates plus the second-use
XORs that remain after second_use_plan folds masks into gates.  A
restriction (--restrict, bit masks of S-box inputs) asks the search for
networks whose gates can take those inputs' key masks (SBOX_RESTRICT in
sbox_synth.cpp); the inputs that matter are the shared ones, 0, 1, 4 and 5.
Run by hand when the search changes; the committed sbox_networks.txt is what
the emitter reads, so a normal build does not search.

    python -m paper_2007_10752_amd.gen.synth_sboxes --restarts 2000 --jobs 8
    python -m paper_2007_10752_amd.gen.synth_sboxes --restarts 1400 --restrict 1,2,16,32
"""
import argparse
import concurrent.futures as cf
import itertools
import os
import subprocess
import tempfile

from .des_tables import SBOX
from .networks import (NETWORKS_PATH, foldable, format_networks, load_networks, parse_network,
                       second_use_plan, verify_network)

HERE = os.path.dirname(os.path.abspath(__file__))


def _build(tmpdir):
    exe = os.path.join(tmpdir, "sbox_synth")
    subprocess.run(["g++", "-O2", "-o", exe, os.path.join(HERE, "sbox_synth.cpp")], check=True)
    return exe


def _run(exe, box, restarts, seed, restrict, lookahead):
    vals = [str(v) for row in SBOX[box] for v in row]
    env = dict(os.environ, SBOX_RESTRICT=str(restrict), SBOX_LOOKAHEAD=str(lookahead))
    r = subprocess.run([exe, str(restarts), str(seed)] + vals, check=True,
                       capture_output=True, text=True, env=env)
    lines = r.stdout.splitlines()
    if not lines or int(lines[0].split()[1]) >= 1 << 20:
        return None  # every restart of this job was dropped
    return parse_network(r.stdout)


def round_cost(nets):
    """Gates plus second-use XORs per round for a full set of networks."""
    _, folded = second_use_plan(nets)
    return sum(len(n["gates"]) for n in nets.values()) + 16 - len(folded)


def _fold_sets(net):
    return frozenset(frozenset(c) for n in range(5) for c in itertools.combinations((0, 1, 4, 5), n)
                     if foldable(net, c))


def choose(cands):
    """Per box, the candidate networks; returns the combination of least
    round_cost (candidates dominated within their box, more gates and no fold
    set the other lacks, are dropped first)."""
    pruned = {}
    for box, nets in cands.items():
        keep = []
        for n in sorted(nets, key=lambda n: len(n["gates"])):
            fs = _fold_sets(n)
            if any(len(k["gates"]) <= len(n["gates"]) and fs <= _fold_sets(k) for k in keep):
                continue
            keep.append(n)
        pruned[box] = keep
    boxes = sorted(pruned)
    best, best_cost = None, None
    for combo in itertools.product(*(pruned[b] for b in boxes)):
        nets = dict(zip(boxes, combo))
        cost = round_cost(nets)
        if best_cost is None or cost < best_cost:
            best, best_cost = nets, cost
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--restarts", type=int, default=1000)
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 4)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--boxes", default="0,1,2,3,4,5,6,7")
    ap.add_argument("--restrict", default="0",
                    help="comma-separated bit masks of restricted inputs, one search each")
    ap.add_argument("--lookahead", type=int, default=int(os.environ.get("SBOX_LOOKAHEAD", "0")))
    args = ap.parse_args()
    boxes = [int(b) for b in args.boxes.split(",")]
    masks = [int(m) for m in args.restrict.split(",")]
    try:
        current = load_networks()
    except FileNotFoundError:
        current = {}
    cands = {b: [current[b]] for b in range(8) if b in current}
    with tempfile.TemporaryDirectory() as td:
        exe = _build(td)
        per_job = max(1, args.restarts // args.jobs)
        with cf.ThreadPoolExecutor(args.jobs) as pool:
            futs = {}
            for box in boxes:
                for mask in masks:
                    for j in range(args.jobs):
                        seed = args.seed * 1000003 + box * 7919 + mask * 104729 + j
                        futs[pool.submit(_run, exe, box, per_job, seed, mask, args.lookahead)] = (box, mask)
            found = {}
            for fut in cf.as_completed(futs):
                box, mask = futs[fut]
                net = fut.result()
                if net is None:
                    continue
                verify_network(box, net)
                key = (box, mask)
                if key not in found or len(net["gates"]) < len(found[key]["gates"]):
                    found[key] = net
    for (box, mask), net in sorted(found.items()):
        print("S%d restrict %d: %d gates" % (box + 1, mask, len(net["gates"])))
        cands.setdefault(box, []).append(net)
    best = choose(cands)
    _, folded = second_use_plan(best)
    for box in sorted(best):
        print("S%d: %d gates" % (box + 1, len(best[box]["gates"])))
    print("round: %d gates + %d XORs (%d second-use masks folded)"
          % (sum(len(n["gates"]) for n in best.values()), 48 - len(folded), len(folded)))
    with open(NETWORKS_PATH, "w") as f:
        f.write(format_networks(best))


if __name__ == "__main__":
    main()
