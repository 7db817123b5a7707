"""Measured MI355X ceilings (through include/tdes_probe.h), timed with HIP
events on the stream the probe kernels run on."""
import ctypes

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
    (256 CUs x 4 SIMDs; a workgroup is 4 waves).  Under rocprofv3 --pmc
    SQ_INSTS_VALU SQ_ACTIVE_INST_VALU2 the share of instructions issued in
    pairs is 2 * SQ_ACTIVE_INST_VALU2 / SQ_INSTS_VALU per dispatch."""
    import json
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for wps in (2, 4, 8):
        blocks = cus * wps  # cus * 4 SIMDs * wps waves / 4 waves per block
        for op in OPS:
            r = valu_rate(op, blocks=blocks, iters=8000 // wps, reps=2)
            print(json.dumps({"op": op, "waves_per_simd": wps, "blocks": blocks,
                              "T_lane_ops_per_s": round(r / 1e12, 2)}), flush=True)
    print(json.dumps({"copy_TBps": round(copy_rate() / 1e12, 3)}), flush=True)


if __name__ == "__main__":
    main()
