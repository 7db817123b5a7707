"""Measured MI355X ceilings (through include/tdes_probe.h), timed with HIP
events on the stream the probe kernels run on.

    python -m paper_2007_10752_amd.probe [--quick] [--ms 50]

By default the shader clock is settled first (0.5 s of the bitop3 probe)
and every figure comes from launches of at least --ms milliseconds
(median of 3): the clock under sustained load, as the cipher kernels see
it.  --quick runs short launches from a cold start instead."""
import argparse
import ctypes
import time

from . import tdes

OPS = {"bitop3": 0, "xor": 1, "xor_sgpr": 2, "perm": 3, "bfi": 4, "lshl": 5, "lshr": 6,
       "add": 7, "bfe": 8}
LANE_OPS_PER_ITER = 16


def valu_rate(op="bitop3", blocks=8192, iters=4000, reps=3):
    """32-bit VALU lane operations per second sustained by the probe."""
    import torch
    sink = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    lib = tdes.lib()

    def launch():
        rc = lib.tdes_probe_valu(OPS[op], ctypes.c_void_p(sink.data_ptr()), blocks, iters,
                                 ctypes.c_void_p(int(stream.cuda_stream)))
        if rc != 0:
            raise RuntimeError("tdes_probe_valu failed: %d" % rc)

    launch()
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        launch()
        b.record(stream)
        b.synchronize()
        t = a.elapsed_time(b) / 1e3
        best = t if best is None else min(best, t)
    return blocks * 256 * LANE_OPS_PER_ITER * iters / best


LDS_MODES = {"consec": 0, "samebank": 1, "bcast": 2, "b128": 3}
LDS_BYTES_PER_READ = {"consec": 4, "samebank": 4, "bcast": 4, "b128": 16}


def _timed(launch, reps, stat=min):
    import torch
    stream = torch.cuda.current_stream()
    launch()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        launch()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    return stat(ts)


def _median(ts):
    return sorted(ts)[len(ts) // 2]


def lds_rate(mode="consec", blocks=512, iters=4000, reps=3, stat=min):
    """LDS bytes read per second by the probe (64 KiB of LDS per workgroup)."""
    import torch
    sink = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    lib = tdes.lib()

    def launch():
        rc = lib.tdes_probe_lds(LDS_MODES[mode], ctypes.c_void_p(sink.data_ptr()), blocks, iters,
                                ctypes.c_void_p(int(stream.cuda_stream)))
        if rc != 0:
            raise RuntimeError("tdes_probe_lds failed: %d" % rc)

    t = _timed(launch, reps, stat)
    return blocks * 256 * 16 * iters * LDS_BYTES_PER_READ[mode] / t


def _sized(rate_fn, target_s, iters0):
    """iters for a launch of about target_s seconds (from a short launch)."""
    t0 = time.perf_counter()
    rate_fn(iters0, 1)
    dt = max(time.perf_counter() - t0, 1e-4)  # two launches: a warm one and the timed one
    return max(iters0, int(iters0 * target_s / (dt / 2)))


def copy_rate(nbytes=1 << 30, reps=5):
    """HBM bytes moved per second (read + write) by the plain copy probe."""
    import torch
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    lib = tdes.lib()

    def launch():
        rc = lib.tdes_probe_copy(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                 nbytes, ctypes.c_void_p(int(stream.cuda_stream)))
        if rc != 0:
            raise RuntimeError("tdes_probe_copy failed: %d" % rc)

    launch()
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        launch()
        b.record(stream)
        b.synchronize()
        t = a.elapsed_time(b) / 1e3
        best = t if best is None else min(best, t)
    return 2 * nbytes / best


def main():
    """Lane-operation rate per probed opcode at 2, 4 and 8 waves per SIMD
    (256 CUs x 4 SIMDs; a workgroup is 4 waves), LDS read rates per pattern
    and the copy rate.  Under rocprofv3 --pmc SQ_INSTS_VALU
    SQ_ACTIVE_INST_VALU2 the share of instructions issued in pairs is
    2 * SQ_ACTIVE_INST_VALU2 / SQ_INSTS_VALU per dispatch; GRBM_GUI_ACTIVE
    over the launch time gives the clock."""
    import json
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="short launches from a cold start")
    ap.add_argument("--ms", type=float, default=50.0, help="launch length when settled")
    args = ap.parse_args()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    if args.quick:
        for wps in (2, 4, 8):
            blocks = cus * wps  # cus * 4 SIMDs * wps waves / 4 waves per block
            for op in OPS:
                r = valu_rate(op, blocks=blocks, iters=8000 // wps, reps=2)
                print(json.dumps({"op": op, "waves_per_simd": wps, "blocks": blocks,
                                  "T_lane_ops_per_s": round(r / 1e12, 2)}), flush=True)
        print(json.dumps({"copy_TBps": round(copy_rate() / 1e12, 3)}), flush=True)
        return
    target = args.ms / 1e3
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.5:  # settle the clock
        valu_rate("bitop3", blocks=cus * 8, iters=20000, reps=1)
    for wps in (4, 8):
        blocks = cus * wps
        for op in OPS:
            iters = _sized(lambda it, r: valu_rate(op, blocks, it, r), target, 2000)
            r = valu_rate(op, blocks=blocks, iters=iters, reps=3)
            print(json.dumps({"op": op, "waves_per_simd": wps, "blocks": blocks, "iters": iters,
                              "ms_per_launch": round(blocks * 256 * 16 * iters / r * 1e3, 2),
                              "T_lane_ops_per_s": round(r / 1e12, 2)}), flush=True)
    # LDS: 64 KiB per workgroup, so at most 2 workgroups (8 waves) per CU
    for mode in LDS_MODES:
        blocks = cus * 2
        iters = _sized(lambda it, r: lds_rate(mode, blocks, it, r), target, 1000)
        r = lds_rate(mode, blocks=blocks, iters=iters, reps=3)
        print(json.dumps({"lds": mode, "blocks": blocks, "iters": iters,
                          "TB_per_s": round(r / 1e12, 2),
                          "bytes_per_clk_per_cu_at_2.4GHz": round(r / cus / 2.4e9, 1)}),
              flush=True)
    print(json.dumps({"copy_TBps": round(copy_rate() / 1e12, 3)}), flush=True)


if __name__ == "__main__":
    main()
