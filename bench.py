#!/usr/bin/env python3
"""Benchmark: 3DES-EDE ECB encryption of 1 GiB (134,217,728 blocks) resident
in HBM on one MI355X, through the library's C ABI.

One step = key schedule of the 3-key bundle (host) + one fused 48-round
encryption launch over the whole buffer.  The GPU's shader clock ramps up
over the first ~60 ms of sustained load, so the step first repeats for
--settle-seconds (the first 10 launches from idle are reported as
settle.cold_first10_GBps); then W untimed warm-up steps, then K timed steps
between device synchronisations.  Every launch is also bracketed by HIP
events on the stream it runs on, which gives the kernel's own average
duration for the roofline figure.  The oracle is timed on the host cores on
a bounded sample of the same input (cpu_baseline).

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GIB = 1 << 30


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kernel", default="bitslice", choices=["bitslice", "spbox"])
    ap.add_argument("--nbytes", type=int, default=GIB, help="payload bytes (default 1 GiB)")
    ap.add_argument("--input", default="uniform", choices=["uniform", "zero", "pattern"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target wall time of the oracle sample (0 disables)")
    ap.add_argument("--batched", type=int, default=1,
                    help="also time the batched form (16,384 log-normal messages); 0 disables")
    ap.add_argument("--settle-seconds", type=float, default=0.3,
                    help="repeat the step this long before the warm-up steps: the shader clock "
                         "ramps up over the first ~60 ms of sustained load (0 disables)")
    ap.add_argument("--modes", type=int, default=1,
                    help="1: also time CTR, CBC decryption and the paper's design on the same 1 GiB")
    ap.add_argument("--host", type=int, default=1,
                    help="1: also time the host-resident form (1 GiB pinned, PCIe included)")
    ap.add_argument("--serve-seconds", type=float, default=1.0,
                    help="length of each open-loop serving run (0 disables serving)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run plain device copies of the same size (for PMC scaling)")
    return ap.parse_args()


def cpu_baseline(key, host, target_s):
    import numpy as np

    import oracle
    threads = oracle.set_threads(0)
    # calibrate on a small slice, then size the sample for ~target_s
    probe = host[: 8 * 16384]
    t0 = time.perf_counter()
    oracle.tdes_ecb(key, probe)
    dt = max(time.perf_counter() - t0, 1e-6)
    nblk = int(16384 * target_s / dt)
    nblk = max(16384, min(nblk, host.size // 8))
    sample = np.ascontiguousarray(host[: 8 * nblk])
    t0 = time.perf_counter()
    oracle.tdes_ecb(key, sample)
    dt = time.perf_counter() - t0
    return {"value": sample.size / dt / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "first %d blocks (%.1f MiB) of the same input, 3DES-ECB encrypt, %.2f s"
                      % (nblk, sample.size / 2**20, dt)}


def time_launches(fn, reps, stream):
    """Median wall time of `reps` calls of fn() between HIP events on stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def batched_section(steps, settle_s=0.3):
    """The batched form on 16,384 messages (log-normal lengths, median 4 KiB,
    sigma 1, 8 B .. 1 MiB; own 3-key bundle each; 50/50 directions), against
    the plain kernel over the same bytes with one key and against one plain
    launch per message."""
    import torch

    from paper_2007_10752_amd import tdes
    from paper_2007_10752_amd import workloads as W
    lay = W.batched_layout(W.SEED_BASE + 3)
    total = lay["total"]
    data = W.uniform_bytes(W.rng(W.SEED_BASE + 3 + W.KEY_SEED_OFFSET), total)
    x = torch.from_numpy(data).cuda()
    out = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    b = tdes.Batch(lay["keys"], lay["offsets"], lay["offsets"], lay["lengths"], lay["dirs"])
    # settle the clock on this workload first (as for the headline)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < settle_s:
        for _ in range(20):
            b.submit(x, out)
        torch.cuda.synchronize()
    mult = b.autotune(x, out, reps=3)
    t_batch = time_launches(lambda: b.submit(x, out), max(3, steps), stream)
    sched = tdes.key_schedule(lay["keys"][0])
    sh = int(stream.cuda_stream)
    t_plain = time_launches(lambda: tdes.ecb_crypt_ptr(sched, 0, 1, x.data_ptr(), out.data_ptr(),
                                                       total, sh), max(3, steps), stream)
    scheds = tdes.key_schedules(lay["keys"])
    offs, lens, dirs = lay["offsets"].tolist(), lay["lengths"].tolist(), lay["dirs"].tolist()
    xb, ob = x.data_ptr(), out.data_ptr()

    def per_message():
        for i in range(len(lens)):
            tdes.ecb_crypt_ptr(scheds[i], dirs[i], 1, xb + offs[i], ob + offs[i], lens[i], sh)

    t_loop = time_launches(per_message, 1, stream)
    # the same batch captured once in a HIP graph and replayed
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.submit(x, out, stream=torch.cuda.current_stream())
    t0 = time.perf_counter()  # the per-message loop above lets the clock fall back
    while time.perf_counter() - t0 < settle_s:
        for _ in range(20):
            graph.replay()
        torch.cuda.synchronize()
    t_graph = time_launches(graph.replay, max(3, steps), stream)
    return {"value": round(total / t_batch / 1e9, 3), "unit": "GB/s",
            "ms": round(t_batch * 1e3, 4), "messages": len(lens), "bytes": total,
            "graph_replay_GBps": round(total / t_graph / 1e9, 3),
            "autotuned_grid_multiplier": mult,
            "plain_same_bytes_GBps": round(total / t_plain / 1e9, 3),
            "per_message_launches_GBps": round(total / t_loop / 1e9, 3),
            "config": "16384 msgs, lognormal median 4 KiB sigma 1, clip 8 B..1 MiB, "
                      "per-message 3-key bundle, 50/50 enc/dec, seed %d" % (W.SEED_BASE + 3)}


def host_section(steps):
    """The host-resident form (PCIe included): 1 GiB of seeded random bytes
    in pinned host memory, encrypted into pinned host memory, directly (the
    kernel on the mapped host buffers) and staged (8 MiB chunks through 3
    device slots); with the copy engines' own rates over the same buffers for
    reference (one direction at a time, and both at once)."""
    import torch

    from paper_2007_10752_amd import tdes
    from paper_2007_10752_amd import workloads as W
    n = GIB
    key = W.key_bundle(W.rng(W.SEED_BASE + 2 + W.KEY_SEED_OFFSET))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(W.SEED_BASE + 4)
    x = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda", generator=gen)
    want = tdes.encrypt(key, x)
    src = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    dst = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    src.copy_(x)
    d = torch.empty_like(x)
    torch.cuda.synchronize()
    reps = max(3, min(steps, 7))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[len(ts) // 2]

    t_direct = timed(lambda: tdes.ecb_host(key, src, dst))
    ok = bool(torch.equal(dst.cuda(), want))
    pipe = tdes.HostPipeline(8 << 20, 3)
    t_staged = timed(lambda: pipe.run(key, src, dst))
    ok = ok and bool(torch.equal(dst.cuda(), want))
    t_h2d = timed(lambda: d.copy_(src, non_blocking=True))
    t_d2h = timed(lambda: dst.copy_(want, non_blocking=True))
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()

    def both():
        with torch.cuda.stream(sa):
            d.copy_(src, non_blocking=True)
        with torch.cuda.stream(sb):
            dst.copy_(want, non_blocking=True)

    t_both = timed(both)
    direct, both_rate = n / t_direct / 1e9, n / t_both / 1e9
    return {"value": round(direct, 2), "unit": "GB/s", "mode": "direct",
            "ms": round(t_direct * 1e3, 3), "bytes": n,
            "staged_GBps": round(n / t_staged / 1e9, 2), "staged_chunk_bytes": 8 << 20,
            "staged_slots": 3,
            "copy_h2d_GBps": round(n / t_h2d / 1e9, 2), "copy_d2h_GBps": round(n / t_d2h / 1e9, 2),
            "copy_both_directions_GBps": round(both_rate, 2),
            "frac_of_copy_both_directions": round(direct / both_rate, 3),
            "equal_to_device_path": ok,
            "config": "1 GiB, pinned host in and out, 3-key, seed %d" % (W.SEED_BASE + 4)}


def serving_section(seconds):
    """Open-loop Poisson request streams at 5k / 20k / 80k requests/s (sizes
    70 % 64 B-1 KiB, 25 % 4-64 KiB, 5 % 1-16 MiB, log-uniform within a band;
    own 3-key bundle each; 50/50 directions; payloads sliced from a 4 GiB
    device pool), served with continuous batching (4 slots, 32 GiB in-flight
    budget) and, as the reference, one plain launch per request in arrival
    order.  Latency runs from each request's scheduled arrival."""
    import torch

    from paper_2007_10752_amd import serve as S
    from paper_2007_10752_amd import workloads as W
    gen = torch.Generator(device="cuda").manual_seed(W.SEED_BASE + 4)
    pool = torch.randint(0, 256, (4 << 30,), dtype=torch.uint8, device="cuda", generator=gen)
    arena_bytes = 16 << 30
    arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device="cuda")
    base = arena.data_ptr() + (-arena.data_ptr()) % 256
    res = {"config": "Poisson arrivals, %.1f s per run, sizes 70%% 64 B-1 KiB / 25%% 4-64 KiB "
                     "/ 5%% 1-16 MiB log-uniform, 3-key bundle and direction per request, "
                     "budget 32 GiB in flight, 4 slots" % seconds}
    for rate in (5000, 20000, 80000):
        trace = W.serving_trace(W.SEED_BASE + 0x500 + rate, rate, seconds)
        reqs = S.make_requests(trace, pool.data_ptr(), pool.numel(), W.SEED_BASE + 0x600 + rate)
        for mode, name in ((S.BATCHED, "batched"), (S.PLAIN, "plain")):
            srv = S.Server(base, arena_bytes, budget_bytes=32 << 30, mode=mode, slots=4,
                           max_batch_msgs=8192)
            # warm-up: the first 200 requests of the trace, replayed untimed
            S.run_open_loop(srv, reqs[:200].copy(), trace["arrival"][:200] - trace["arrival"][0])
            lat, status, wall, st = S.run_open_loop(srv, reqs, trace["arrival"], timeout_s=120)
            srv.close()
            r = S.summarize(lat, trace["size"], wall, st, rate, seconds)
            r["errors"] = int((status != 0).sum())
            res["%s_%dk" % (name, rate // 1000)] = r
            print("serve", name, rate, r["p50_ms"], r["p99_ms"], r["GBps"], file=sys.stderr,
                  flush=True)
    del pool, arena
    return res


def traffic_from_profile(kernel, nbytes):
    """HBM bytes per launch from the committed PMC summary, if it was taken
    on the current kernel source and workload; else None."""
    path = os.path.join(ROOT, "profiles", "%s_1gib_pmc.md" % kernel)
    if not os.path.exists(path) or nbytes != GIB:
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("bench-traffic:"):
                for kv in line.split(":", 1)[1].split():
                    k, v = kv.split("=")
                    fields[k] = v
    if fields.get("source_sha256") != kernel_source_hash(kernel):
        return None
    return float(fields["bytes_per_launch"])


def kernel_source_hash(kernel):
    """Hash of the sources a kernel is compiled from (to tell whether stored
    counter readings still describe it)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2007_10752_amd", "csrc")
    files = {"bitslice": ["bitslice.hip", "bitslice_core.h", "lds_masks.h",
                          "generated/bitslice_gen.h"],
             "spbox": ["spbox.hip", "generated/spbox_gen.h"]}[kernel]
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: ECB needs no exchange between GPUs, and this "
              "build runs on a single MI355X (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2007_10752_amd import costs
    from paper_2007_10752_amd import tdes
    from paper_2007_10752_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    nbytes = args.nbytes
    assert nbytes % 8 == 0
    key = W.key_bundle(W.rng(W.SEED_BASE + 2 + W.KEY_SEED_OFFSET))
    if args.input == "uniform":
        host = W.uniform_bytes(W.rng(W.SEED_BASE + 2), nbytes)
    elif args.input == "zero":
        host = np.zeros(nbytes, np.uint8)
    else:
        host = W.pattern_bytes(nbytes)
    x = torch.from_numpy(host).cuda()
    out = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    kernel = tdes.KERNELS[args.kernel]

    def step():
        sched = tdes.key_schedule(key)
        tdes.ecb_crypt_ptr(sched, tdes.ENCRYPT, kernel, x.data_ptr(), out.data_ptr(), nbytes, sh)

    # From idle: the first launches run while the clock ramps up (reported
    # as cold_first10_GBps, not the value).
    step()
    torch.cuda.synchronize()
    cold = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(10)]
    for a, b in cold:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    cold_s = sum(a.elapsed_time(b) for a, b in cold) / len(cold) / 1e3
    # Settle: the same step, repeated until the clock has ramped up.
    t_settle = time.perf_counter()
    n_settle = 0
    while time.perf_counter() - t_settle < args.settle_seconds:
        for _ in range(10):
            step()
        n_settle += 10
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("warmup done (%d settle steps)" % n_settle, file=sys.stderr, flush=True)

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in ev]
    avg_kernel_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    print("timed %d steps: %.3f ms/step" % (args.steps, wall / args.steps * 1e3),
          file=sys.stderr, flush=True)

    if args.copy_calibration:
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del y

    nblocks = nbytes // 8
    value = nbytes * args.steps / wall / 1e9
    ops = costs.ops_per_block(args.kernel) * nblocks
    achieved = ops / avg_kernel_s
    traffic = traffic_from_profile(args.kernel, nbytes)
    line = {
        "metric": "3DES-ECB GB/s at 1 GiB (bit-exact); batched/served GB/s + p50/p99 vs plain",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "settle": {"seconds": args.settle_seconds, "steps": n_settle,
                   "cold_first10_GBps": round(nbytes / cold_s / 1e9, 3)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "3des-ede-ecb-encrypt", "bytes": nbytes, "blocks": nblocks,
                   "input": args.input, "key": "3-key", "kernel": args.kernel,
                   "seed": W.SEED_BASE + 2},
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved / 1e12, 3),
            "peak": round(costs.VALU_PEAK_OPS / 1e12, 3),
            "unit": "T lane-ops/s (32-bit VALU)",
            "frac": round(achieved / costs.VALU_PEAK_OPS, 4),
            "traffic": traffic,
            "ops_per_block": round(costs.ops_per_block(args.kernel), 2),
            "kernel_ms": round(avg_kernel_s * 1e3, 4),
            "hbm_gbps": round(costs.HBM_BYTES_PER_BLOCK * nblocks / avg_kernel_s / 1e9, 2),
            "hbm_frac": round(costs.HBM_BYTES_PER_BLOCK * nblocks / avg_kernel_s
                              / costs.HBM_PEAK_BYTES, 4),
        },
    }
    if args.modes:
        iv = W.uniform_bytes(W.rng(W.SEED_BASE + 5), 8)
        sched = tdes.key_schedule(key)
        t_ctr = time_launches(lambda: tdes.ctr_crypt_ptr(sched, iv, x.data_ptr(), out.data_ptr(),
                                                         nbytes, sh), max(3, args.steps), stream)
        line["ctr"] = {"value": round(nbytes / t_ctr / 1e9, 3), "unit": "GB/s",
                       "ms": round(t_ctr * 1e3, 4),
                       "config": "same bytes and key in CTR mode, seeded 8-byte IV"}
        t_cbc = time_launches(lambda: tdes.cbc_decrypt_ptr(sched, iv, x.data_ptr(),
                                                           out.data_ptr(), nbytes, sh),
                              max(3, args.steps), stream)
        line["cbc_decrypt"] = {"value": round(nbytes / t_cbc / 1e9, 3), "unit": "GB/s",
                               "ms": round(t_cbc * 1e3, 4),
                               "config": "same bytes and key, CBC decryption, seeded 8-byte IV"}
        t_paper = time_launches(lambda: tdes.paper_design_ptr(sched, tdes.ENCRYPT, x.data_ptr(),
                                                               out.data_ptr(), nbytes, sh),
                                3, stream)
        line["paper_design"] = {"value": round(nbytes / t_paper / 1e9, 3), "unit": "GB/s",
                                "ms": round(t_paper * 1e3, 3),
                                "config": "same bytes and key, ECB encrypt with the paper's "
                                          "one-thread-per-bit design (three launches)"}
        print("modes done", file=sys.stderr, flush=True)
    del x, out
    torch.cuda.empty_cache()
    if args.batched:
        line["batched"] = batched_section(args.steps, args.settle_seconds)
        print("batched done", file=sys.stderr, flush=True)
    if args.host:
        line["host_resident"] = host_section(args.steps)
        print("host-resident done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if args.serve_seconds > 0:
        line["served"] = serving_section(args.serve_seconds)
    if args.cpu_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(key, host, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
