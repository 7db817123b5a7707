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
a bounded sample of the same input (cpu_baseline), and the timed run's
output is checked against the oracle: the whole 1 GiB by SHA-256 against a
digest the oracle wrote (tests/golden), and block by block on the sample.

Beside the headline, the other workloads are reported in their own
objects: 32 KiB encrypt and decrypt (launch-bound), 64 MiB with 3-key and
2-key bundles in both directions on both kernels, 1 GiB of all-zero and
repeating-pattern input, the batched form (16,384 messages: a stream of
batches over two streams, one stream, one submit alone, and from raw key
bundles), the host-resident form and the request server.

Prints one JSON line.
"""
import argparse
import hashlib
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
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="length of each open-loop serving run (0 disables serving)")
    ap.add_argument("--serve-warmup", type=float, default=1.0,
                    help="length of the warm-up run before each serving run")
    ap.add_argument("--configs", type=int, default=1,
                    help="1: also time 32 KiB, the 64 MiB matrix and the structured 1 GiB inputs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run plain device copies of the same size (for PMC scaling)")
    return ap.parse_args()


def cpu_baseline(key, host, target_s, gpu_out_prefix=None):
    """The oracle on the host cores: all threads on the first N blocks of the
    headline input (N sized for ~target_s), one thread on a sample sized for
    ~target_s / 3, and medians of 3 runs on the 32 KiB and 64 MiB workloads
    (all threads).  The all-thread sample's output is compared block by block
    with the GPU's output for the same blocks (gpu_out_prefix)."""
    import numpy as np

    import oracle
    from paper_2007_10752_amd import workloads as W
    threads = oracle.set_threads(0)

    def sized(seconds, nmax):
        probe = host[: 8 * 16384]
        t0 = time.perf_counter()
        oracle.tdes_ecb(key, probe)
        dt = max(time.perf_counter() - t0, 1e-6)
        return max(16384, min(int(16384 * seconds / dt), nmax))

    nmax = host.size // 8
    if gpu_out_prefix is not None:
        nmax = min(nmax, gpu_out_prefix.size // 8)
    nblk = sized(target_s, nmax)
    sample = np.ascontiguousarray(host[: 8 * nblk])
    t0 = time.perf_counter()
    want = oracle.tdes_ecb(key, sample)
    dt = time.perf_counter() - t0
    res = {"value": sample.size / dt / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": "first %d blocks (%.1f MiB) of the same input, 3DES-ECB encrypt, %.2f s"
                     % (nblk, sample.size / 2**20, dt)}
    if gpu_out_prefix is not None:
        eq = (want.reshape(-1, 8) == gpu_out_prefix[: sample.size].reshape(-1, 8)).all(axis=1)
        res["bit_exact_blocks"] = int(eq.sum())
        res["blocks_compared"] = int(eq.size)
    del want
    # one thread
    oracle.set_threads(1)
    n1 = sized(target_s / 3, host.size // 8)
    s1 = np.ascontiguousarray(host[: 8 * n1])
    t0 = time.perf_counter()
    oracle.tdes_ecb(key, s1)
    d1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    res["one_thread"] = {"value": s1.size / d1 / 1e9, "unit": "GB/s", "cores": 1,
                         "sample": "first %d blocks (%.1f MiB), %.2f s" % (n1, s1.size / 2**20, d1)}

    def median3(data, k):
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.tdes_ecb(k, data)
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[1]

    c1 = W.uniform_bytes(W.rng(W.SEED_BASE + 0), 4096 * 8)
    k1 = W.key_bundle(W.rng(W.SEED_BASE + 0 + W.KEY_SEED_OFFSET))
    t = median3(c1, k1)
    res["c1_32kib"] = {"value": c1.size / t / 1e9, "unit": "GB/s", "ms": t * 1e3,
                       "cores": threads, "runs": 3, "stat": "median"}
    c2 = W.uniform_bytes(W.rng(W.SEED_BASE + 1), 64 << 20)
    k2 = W.key_bundle(W.rng(W.SEED_BASE + 1 + W.KEY_SEED_OFFSET))
    t = median3(c2, k2)
    res["c2_64mib"] = {"value": c2.size / t / 1e9, "unit": "GB/s", "ms": t * 1e3,
                       "cores": threads, "runs": 3, "stat": "median"}
    return res


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


def settle(fn, seconds):
    """Repeat fn until `seconds` have passed (lets the shader clock ramp up)."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()


def frac_of_peak(kernel, nbytes, seconds):
    from paper_2007_10752_amd import costs
    return round(costs.ops_per_block(kernel) * (nbytes // 8) / seconds / costs.VALU_PEAK_OPS, 4)


def c1_section():
    """32 KiB (4,096 blocks) encrypt, then decrypt of the result: the
    launch-bound case, through the library's automatic kernel choice (the
    table kernel at this size: one block per lane has the shorter path
    through the 48 rounds), with the bitsliced kernel beside it.  Median of
    200 launches each, timed with HIP events on the stream (kernel plus
    launch gap as the GPU sees it), and the host rate of back-to-back calls
    (key schedule + launch, one sync at the end).  Both ciphertexts are
    checked against the oracle, the round trip against the input."""
    import numpy as np
    import torch

    import oracle
    from paper_2007_10752_amd import tdes
    from paper_2007_10752_amd import workloads as W
    data = W.uniform_bytes(W.rng(W.SEED_BASE + 0), 4096 * 8)
    key = W.key_bundle(W.rng(W.SEED_BASE + 0 + W.KEY_SEED_OFFSET))
    x = torch.from_numpy(data).cuda()
    ct, pt, ct_bs = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    sched = tdes.key_schedule(key)
    n = x.numel()

    def run(kernel, direction, src, dst):
        return lambda: tdes.ecb_crypt_ptr(sched, direction, kernel, src.data_ptr(), dst.data_ptr(),
                                          n, sh)

    enc = run(tdes.KERNEL_AUTO, tdes.ENCRYPT, x, ct)
    dec = run(tdes.KERNEL_AUTO, tdes.DECRYPT, ct, pt)
    enc_bs = run(tdes.KERNEL_BITSLICE, tdes.ENCRYPT, x, ct_bs)
    settle(enc, 0.05)
    t_enc = time_launches(enc, 200, stream)
    t_dec = time_launches(dec, 200, stream)
    t_enc_bs = time_launches(enc_bs, 200, stream)
    torch.cuda.synchronize()
    reps = 500
    t0 = time.perf_counter()
    for _ in range(reps):
        tdes.ecb_crypt_ptr(tdes.key_schedule(key), tdes.ENCRYPT, tdes.KERNEL_AUTO, x.data_ptr(),
                           ct.data_ptr(), n, sh)
    torch.cuda.synchronize()
    t_host = (time.perf_counter() - t0) / reps
    want = oracle.tdes_ecb(key, data)
    ok = bool(np.array_equal(ct.cpu().numpy(), want)) and \
        bool(np.array_equal(ct_bs.cpu().numpy(), want)) and bool(torch.equal(pt, x))
    return {"encrypt_GBps": round(n / t_enc / 1e9, 3), "encrypt_us": round(t_enc * 1e6, 2),
            "decrypt_GBps": round(n / t_dec / 1e9, 3), "decrypt_us": round(t_dec * 1e6, 2),
            "host_calls_GBps": round(n / t_host / 1e9, 3),
            "host_us_per_call": round(t_host * 1e6, 2),
            "frac": frac_of_peak("spbox", n, t_enc),
            "kernel": "automatic choice: %s" % tdes.auto_kernel(n),
            "bitsliced_encrypt_us": round(t_enc_bs * 1e6, 2),
            "bitsliced_encrypt_GBps": round(n / t_enc_bs / 1e9, 3),
            "bit_exact_vs_oracle_and_round_trip": ok, "launches": 200, "stat": "median",
            "config": "4096 blocks (32 KiB) uniform, 3-key bundle, seed %d" % (W.SEED_BASE + 0)}


def c2_section(steps):
    """64 MiB (8,388,608 blocks) of uniform bytes, 3-key and 2-key (K3 = K1)
    bundles, encrypt and decrypt, on the bitsliced and the table kernel:
    median of max(20, steps) launches each, after the clock has settled on
    that kernel.  Each result is checked against the other kernel's, and
    decryption of the encryption against the input."""
    import torch

    from paper_2007_10752_amd import tdes
    from paper_2007_10752_amd import workloads as W
    n = 64 << 20
    data = W.uniform_bytes(W.rng(W.SEED_BASE + 1), n)
    kg = W.rng(W.SEED_BASE + 1 + W.KEY_SEED_OFFSET)
    keys = {"3-key": W.key_bundle(kg), "2-key": W.key_bundle(kg, two_key=True)}
    x = torch.from_numpy(data).cuda()
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    outs = {}
    res = {"config": "8388608 blocks (64 MiB) uniform, seed %d; 3-key and 2-key (K3 = K1) "
                     "bundles, key seed %d" % (W.SEED_BASE + 1, W.SEED_BASE + 1 + W.KEY_SEED_OFFSET),
           "launches": max(20, steps), "stat": "median"}
    for kname in ("bitslice", "spbox"):
        kern = tdes.KERNELS[kname]
        for kt, key in keys.items():
            sched = tdes.key_schedule(key)
            for dname, d in (("encrypt", tdes.ENCRYPT), ("decrypt", tdes.DECRYPT)):
                out = torch.empty_like(x)

                def run(sched=sched, d=d, out=out, kern=kern):
                    tdes.ecb_crypt_ptr(sched, d, kern, x.data_ptr(), out.data_ptr(), n, sh)

                settle(run, 0.1)
                t = time_launches(run, max(20, steps), stream)
                outs[(kname, kt, dname)] = out
                res["%s_%s_%s" % (kname, kt, dname)] = {
                    "GBps": round(n / t / 1e9, 3), "ms": round(t * 1e3, 4),
                    "frac": frac_of_peak(kname, n, t)}
    same = all(torch.equal(outs[("bitslice", kt, dn)], outs[("spbox", kt, dn)])
               for kt in keys for dn in ("encrypt", "decrypt"))
    rt = True
    for kt, key in keys.items():
        back = torch.empty_like(x)
        tdes.ecb_crypt_ptr(tdes.key_schedule(key), tdes.DECRYPT, 1,
                           outs[("bitslice", kt, "encrypt")].data_ptr(), back.data_ptr(), n, sh)
        rt = rt and bool(torch.equal(back, x))
    res["kernels_agree"] = bool(same)
    res["round_trip"] = rt
    return res


def structured_section(x, out, steps):
    """1 GiB of all-zero and of repeating 8-byte pattern input (x and out are
    1 GiB device buffers; x is overwritten), 3-key bundle, both kernels:
    median of max(10, steps) launches.  Every output block must equal the
    oracle's encryption of the one distinct input block."""
    import numpy as np
    import torch

    import oracle
    from paper_2007_10752_amd import tdes
    from paper_2007_10752_amd import workloads as W
    key = W.key_bundle(W.rng(W.SEED_BASE + 2 + W.KEY_SEED_OFFSET))
    sched = tdes.key_schedule(key)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    n = x.numel()
    res = {"config": "1 GiB, 3-key bundle (headline key), all-zero and bytes 01..08 repeated",
           "launches": max(10, steps), "stat": "median"}
    for name, block in (("zero", bytes(8)), ("pattern", bytes(range(1, 9)))):
        x.view(-1, 8).copy_(torch.tensor(list(block), dtype=torch.uint8, device=x.device))
        want = torch.from_numpy(oracle.tdes_ecb(key, np.frombuffer(block, np.uint8))).cuda()
        for kname in ("bitslice", "spbox"):
            kern = tdes.KERNELS[kname]

            def run(kern=kern):
                tdes.ecb_crypt_ptr(sched, tdes.ENCRYPT, kern, x.data_ptr(), out.data_ptr(), n, sh)

            settle(run, 0.2)
            t = time_launches(run, max(10, steps), stream)
            ok = bool((out.view(-1, 8) == want).all().item())
            res["%s_%s" % (name, kname)] = {"GBps": round(n / t / 1e9, 3),
                                            "ms": round(t * 1e3, 4),
                                            "frac": frac_of_peak(kname, n, t),
                                            "every_block_equals_oracle": ok}
    return res


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
    tuned = b.autotune(x, out, reps=3)
    t_single = time_launches(lambda: b.submit(x, out), max(3, steps), stream)
    sched = tdes.key_schedule(lay["keys"][0])
    sh = int(stream.cuda_stream)
    t_plain = time_launches(lambda: tdes.ecb_crypt_ptr(sched, 0, 1, x.data_ptr(), out.data_ptr(),
                                                       total, sh), max(3, steps), stream)
    # A stream of batches, as a server runs them: back-to-back submits,
    # alternating between two streams, each batch with its own workspace and
    # output, so that the last waves of one batch share the GPU with the
    # first of the next.  Also on one stream, and the plain kernel on the
    # same bytes the same two ways.
    b2 = tdes.Batch(lay["keys"], lay["offsets"], lay["offsets"], lay["lengths"], lay["dirs"])
    out2 = torch.empty_like(x)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def batch_on(bb, o, st):
        return lambda: bb.submit(x, o, stream=st)

    def plain_on(o, st):
        return lambda: tdes.ecb_crypt_ptr(sched, 0, 1, x.data_ptr(), o.data_ptr(), total,
                                          int(st.cuda_stream))

    def stream_of(fns, k):
        def one():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(k):
                fns[i % len(fns)]()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / k
        # the batch set-up above leaves the GPU idle long enough for the
        # clock to fall back: settle on this loop first
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < settle_s:
            one()
        return sorted(one() for _ in range(3))[1]

    k_stream = max(20, steps)
    lanes = [batch_on(b, out, s1), batch_on(b2, out2, s2)]
    t_one_stream = stream_of(lanes[:1], k_stream)  # the single-submit tuning
    # the configuration for two streams: the autotuner timing the stream of
    # batches over the same two streams
    tuned2 = b.autotune_streams(x, [out, out2], [s1, s2], reps=3)
    t_batch = stream_of(lanes, k_stream)
    t_plain2 = stream_of([plain_on(out, s1), plain_on(out2, s2)], k_stream)
    b.submit(x, out)
    b2.submit(x, out2, stream=stream)
    streams_equal = bool(torch.equal(out, out2))
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
    raw = raw_keys_variant(b, lay, x, out, steps, settle_s)
    return {"value": round(total / t_batch / 1e9, 3), "unit": "GB/s",
            "ms": round(t_batch * 1e3, 4), "messages": len(lens), "bytes": total,
            "value_is": "%d back-to-back batches alternating over two streams, wall time per "
                        "batch (median of 3 runs)" % k_stream,
            "one_stream_GBps": round(total / t_one_stream / 1e9, 3),
            "single_submit_GBps": round(total / t_single / 1e9, 3),
            "single_submit_ms": round(t_single * 1e3, 4),
            "two_streams_outputs_equal": streams_equal,
            "graph_replay_GBps": round(total / t_graph / 1e9, 3),
            "autotuned": {"kmax": tuned["kmax"], "waves_per_simd": tuned["waves"],
                          "grid_multiplier": tuned["grid_mult"], "saved": tuned["saved"]},
            "autotuned_two_streams": {"kmax": tuned2["kmax"], "waves_per_simd": tuned2["waves"],
                                      "grid_multiplier": tuned2["grid_mult"],
                                      "saved": tuned2["saved"]},
            "plain_same_bytes_GBps": round(total / t_plain / 1e9, 3),
            "plain_same_bytes_two_streams_GBps": round(total / t_plain2 / 1e9, 3),
            "per_message_launches_GBps": round(total / t_loop / 1e9, 3),
            "from_raw_keys": raw,
            "config": "16384 msgs, lognormal median 4 KiB sigma 1, clip 8 B..1 MiB, "
                      "per-message 3-key bundle, 50/50 enc/dec, seed %d" % (W.SEED_BASE + 3)}


def raw_keys_variant(b, lay, x, out, steps, settle_s):
    """The batch started from raw 24-byte key bundles, two ways: on the
    device (bundles copied to the GPU, tdes_schedule_expand, submit; one
    stream, timed with HIP events) and on the host (one tdes_key_schedule
    call per bundle from Python, tdes_schedule_upload, submit; wall time to
    completion).  Both must give the precomputed-schedule batch's output."""
    import numpy as np
    import torch

    from paper_2007_10752_amd import tdes
    n, total = b.n_msgs, lay["total"]
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    want = out.clone()
    keys_h = torch.from_numpy(np.ascontiguousarray(lay["keys"]).reshape(-1)).pin_memory()
    keys_d = torch.empty(keys_h.numel(), dtype=torch.uint8, device="cuda")
    sched_d = torch.empty_like(b.sched)

    def submit(sched_ptr):
        tdes.batch_submit_ptr(b.msgs.data_ptr(), n, sched_ptr, n, x.data_ptr(), x.numel(),
                              out.data_ptr(), out.numel(), b.ws.data_ptr(), b.ws_bytes, sh)

    def device_path():
        keys_d.copy_(keys_h, non_blocking=True)
        tdes.schedule_expand(keys_d.data_ptr(), n, sched_d.data_ptr(), sh)
        submit(sched_d.data_ptr())

    settle(device_path, settle_s)
    t_dev = time_launches(device_path, max(3, steps), stream)
    ok_dev = bool(torch.equal(out, want))
    t_expand = time_launches(lambda: tdes.schedule_expand(keys_d.data_ptr(), n, sched_d.data_ptr(),
                                                          sh), max(3, steps), stream)
    sched_h = torch.empty_like(b.sched)
    t_host, t_keys = [], []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sc = tdes.key_schedules(lay["keys"])
        tdes.schedule_upload(sc, sched_h.data_ptr(), sh)
        t1 = time.perf_counter()
        submit(sched_h.data_ptr())
        torch.cuda.synchronize()
        t_host.append(time.perf_counter() - t0)
        t_keys.append(t1 - t0)
    t_host, t_keys = sorted(t_host)[1], sorted(t_keys)[1]
    ok_host = bool(torch.equal(out, want))
    return {"device_GBps": round(total / t_dev / 1e9, 3), "device_ms": round(t_dev * 1e3, 4),
            "expand_kernel_ms": round(t_expand * 1e3, 4),
            "host_GBps": round(total / t_host / 1e9, 3), "host_ms": round(t_host * 1e3, 3),
            "host_schedule_and_upload_ms": round(t_keys * 1e3, 3),
            "equal_to_precomputed": ok_dev and ok_host,
            "config": "device: 393,216 B of bundles copied in, schedule expansion, submit "
                      "(HIP events, median); host: tdes_key_schedule per bundle from Python, "
                      "tdes_schedule_upload, submit (wall, median of 3)"}


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


def serving_section(seconds, warmup_s=1.0):
    """Open-loop Poisson request streams (sizes 70 % 64 B-1 KiB, 25 %
    4-64 KiB, 5 % 1-16 MiB, log-uniform within a band; own 3-key bundle
    each; 50/50 directions; payloads sliced from a 4 GiB device pool), served
    with continuous batching (4 slots, 32 GiB in-flight budget) and, as the
    reference, one plain launch per request in arrival order.  Latency runs
    from each request's scheduled arrival.  Each measured run follows a
    warm-up run of warmup_s on a server of its own, so its counters cover
    the measured requests only.  Rates 5k, 20k and 80k requests/s run in
    both modes; 160k and 320k in batched mode (one plain launch per request
    falls behind already at 80k).  The capacity runs submit a fixed set of
    requests at once (the standard mix, and a mix of 1-16 MiB requests
    only) and report the served rate in each mode."""
    import numpy as np
    import torch

    from paper_2007_10752_amd import serve as S
    from paper_2007_10752_amd import workloads as W
    gen = torch.Generator(device="cuda").manual_seed(W.SEED_BASE + 4)
    pool = torch.randint(0, 256, (4 << 30,), dtype=torch.uint8, device="cuda", generator=gen)
    arena_bytes = 16 << 30
    arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device="cuda")
    base = arena.data_ptr() + (-arena.data_ptr()) % 256

    def server(mode):
        return S.Server(base, arena_bytes, budget_bytes=32 << 30, mode=mode, slots=4,
                        max_batch_msgs=8192)

    res = {"config": "Poisson arrivals, %.1f s per run after a %.1f s warm-up run, sizes 70%% "
                     "64 B-1 KiB / 25%% 4-64 KiB / 5%% 1-16 MiB log-uniform, 3-key bundle and "
                     "direction per request, budget 32 GiB in flight, 4 slots"
                     % (seconds, warmup_s)}
    modes = ((S.BATCHED, "batched"), (S.PLAIN, "plain"))
    for rate in (5000, 20000, 80000, 160000, 320000):
        trace = W.serving_trace(W.SEED_BASE + 0x500 + rate, rate, seconds)
        reqs = S.make_requests(trace, pool.data_ptr(), pool.numel(), W.SEED_BASE + 0x600 + rate)
        warm = W.serving_trace(W.SEED_BASE + 0x700 + rate, rate, warmup_s)
        wreqs = S.make_requests(warm, pool.data_ptr(), pool.numel(), W.SEED_BASE + 0x800 + rate)
        for mode, name in modes if rate <= 80000 else modes[:1]:
            srv = server(mode)
            S.run_open_loop(srv, wreqs, warm["arrival"], timeout_s=120)
            srv.close()
            srv = server(mode)
            lat, status, wall, st = S.run_open_loop(srv, reqs, trace["arrival"], timeout_s=300)
            srv.close()
            r = S.summarize(lat, trace["size"], wall, st, rate, seconds)
            r["errors"] = int((status != 0).sum())
            res["%s_%dk" % (name, rate // 1000)] = r
            print("serve", name, rate, r["p50_ms"], r["p99_ms"], r["GBps"], file=sys.stderr,
                  flush=True)
    # capacity: every request submitted at once
    large = ((1.0, 1 << 20, 16 << 20),)
    for mix, bands, n in (("standard", W.SIZE_BANDS, 100000), ("large", large, 2000)):
        # ~1.25 n arrivals in 1 s, cut to n; the arrival times are not used
        trace = W.serving_trace(W.SEED_BASE + 0x900 + n, 1.25 * n, 1.0, bands=bands)
        trace = {k: v[:n] for k, v in trace.items()}
        n = len(trace["size"])
        reqs = S.make_requests(trace, pool.data_ptr(), pool.numel(), W.SEED_BASE + 0xA00 + n)
        arrival = np.zeros(n)
        for mode, name in modes:
            srv = server(mode)
            S.run_open_loop(srv, reqs[: n // 10], arrival[: n // 10], timeout_s=120)
            srv.close()
            srv = server(mode)
            lat, status, wall, st = S.run_open_loop(srv, reqs, arrival, timeout_s=300)
            srv.close()
            total = float(np.sum(trace["size"]))
            res["capacity_%s_%s" % (mix, name)] = {
                "requests": n, "GBps": round(total / wall / 1e9, 3),
                "requests_per_s": round(n / wall, 1), "wall_s": round(wall, 4),
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "batches": st["batches"],
                "mean_batch": round(st["batched_msgs"] / max(1, st["batches"]), 2),
                "errors": int((status != 0).sum())}
            print("capacity", mix, name, res["capacity_%s_%s" % (mix, name)]["GBps"],
                  file=sys.stderr, flush=True)
    del pool, arena
    return res


def pmc_from_profile(kernel, nbytes):
    """Per-launch counter figures from the committed PMC summary, if it was
    taken on the current kernel source and the 1 GiB workload: HBM bytes
    (bytes_per_launch, scaled by a copy of known size) and VALU wave
    instructions (valu_insts_per_launch).  Empty if there is none."""
    path = os.path.join(ROOT, "profiles", "%s_1gib_pmc.md" % kernel)
    if not os.path.exists(path) or nbytes != GIB:
        return {}
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("bench-pmc:") or line.startswith("bench-traffic:"):
                for kv in line.split(":", 1)[1].split():
                    k, v = kv.split("=")
                    fields[k] = v
    if fields.get("source_sha256") != kernel_source_hash(kernel):
        return {}
    return {k: float(v) for k, v in fields.items() if k != "source_sha256"}


def full_output_check(args, host, out_h, key):
    """SHA-256 of the whole output against the oracle's digest of the same
    workload (tests/golden/ecb_1gib_digest.txt, written by a script that
    calls only the oracle), when the run is that workload."""
    from paper_2007_10752_amd import workloads as W
    path = os.path.join(ROOT, "tests", "golden", "ecb_1gib_digest.txt")
    res = {"full_output_sha256_equals_oracle": None}
    if args.input != "uniform" or args.kernel not in ("bitslice", "spbox") or \
            not os.path.exists(path):
        return res
    d = {}
    with open(path) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#"):
                k, v = ln.split()
                d[k] = v
    if int(d["nbytes"]) != host.size or int(d["data_seed"]) != W.SEED_BASE + 2 or \
            d["key24"] != bytes(key).hex():
        return res
    if hashlib.sha256(memoryview(host)).hexdigest() != d["input_sha256"]:
        res["note"] = "input differs from the digest's"
        return res
    res["full_output_sha256_equals_oracle"] = \
        hashlib.sha256(memoryview(out_h)).hexdigest() == d["encrypt_sha256"]
    res["full_output_blocks"] = int(host.size // 8)
    return res


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

    # The timed run's output against the oracle: the whole buffer by SHA-256
    # against the oracle's digest, and block by block on the cpu_baseline
    # sample (below).
    out_h = out.cpu().numpy()
    bit_exact = full_output_check(args, host, out_h, key)
    print("output checked: %s" % bit_exact, file=sys.stderr, flush=True)

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
    pmc = pmc_from_profile(args.kernel, nbytes)
    traffic = pmc.get("bytes_per_launch")
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
        "bit_exact": bit_exact,
    }
    if "valu_insts_per_launch" in pmc:
        # issued lane operations (wave instructions x 64) over the same time
        issued = pmc["valu_insts_per_launch"] * 64 / avg_kernel_s
        line["roofline"]["issued"] = round(issued / 1e12, 3)
        line["roofline"]["issued_frac"] = round(issued / costs.VALU_PEAK_OPS, 4)
    else:
        line["roofline"]["issued_frac"] = None
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
    if args.configs and nbytes == GIB:
        line["c3_structured"] = structured_section(x, out, args.steps)
        print("structured inputs done", file=sys.stderr, flush=True)
    del x, out
    torch.cuda.empty_cache()
    if args.configs:
        line["c2_64mib"] = c2_section(args.steps)
        print("64 MiB matrix done", file=sys.stderr, flush=True)
        line["c1_32kib"] = c1_section()
        print("32 KiB done", file=sys.stderr, flush=True)
    if args.batched:
        line["batched"] = batched_section(args.steps, args.settle_seconds)
        print("batched done", file=sys.stderr, flush=True)
    if args.host:
        line["host_resident"] = host_section(args.steps)
        print("host-resident done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if args.serve_seconds > 0:
        line["served"] = serving_section(args.serve_seconds, args.serve_warmup)
    if args.cpu_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(key, host, args.cpu_seconds, out_h)
        if "bit_exact_blocks" in line["cpu_baseline"]:
            line["bit_exact"]["oracle_sample_blocks_equal"] = \
                line["cpu_baseline"]["bit_exact_blocks"]
            line["bit_exact"]["oracle_sample_blocks"] = line["cpu_baseline"]["blocks_compared"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
