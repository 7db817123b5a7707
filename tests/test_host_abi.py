"""Host-side checks of the library: no GPU work is done here.

* libtdes.so loads and exports every function include/tdes.h declares;
* the library's key schedule equals the oracle's;
* argument errors are reported before any device call;
* the library's transcription of the Appendix A tables equals the oracle's;
* the S-box networks are exhaustively right (against the oracle's S-boxes);
* the committed generated headers are what the generator writes;
* a CPU emulation of both kernels' arithmetic (from those headers) matches
  the oracle.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2007_10752_amd import tdes as T
from paper_2007_10752_amd import workloads as W
from paper_2007_10752_amd.gen import des_tables as DT
from paper_2007_10752_amd.gen import emit
from paper_2007_10752_amd.gen.networks import MASK_BASE, evaluate, load_networks

import emulate_kernels as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for h in sorted(os.listdir(inc)):
        if h.endswith(".h"):
            text = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, h)).read(), flags=re.S)
            names |= set(re.findall(r"\b(tdes_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = T.lib()
    declared = _header_functions()
    assert declared, "no functions found in tdes.h"
    assert sorted(T.SYMBOLS) == declared
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.tdes_abi_version() == 3


@pytest.mark.parametrize("seed", range(8))
def test_key_schedule_matches_oracle(seed):
    key = W.key_bundle(W.rng(W.SEED_BASE + 0xB00 + seed))
    got = T.key_schedule(key).round_keys()
    for b in range(3):
        assert got[b] == oracle.key_schedule(key[8 * b: 8 * b + 8])


def _crypt(nbytes, d_in=0x1000, d_out=0x100000, dir=0, kernel=0, sched=True):
    s = T.key_schedule(bytes(24))
    lib = T.lib()
    return lib.tdes_ecb_crypt(ctypes.byref(s) if sched else None, dir, kernel,
                              ctypes.c_void_p(d_in), ctypes.c_void_p(d_out),
                              ctypes.c_size_t(nbytes), ctypes.c_void_p(0))


def test_argument_errors_before_device_work():
    # None of these reaches a HIP call (the addresses are never touched).
    assert _crypt(12) == -2                       # TDES_ERR_LENGTH
    assert _crypt(8, d_in=0x1004) == -3           # TDES_ERR_ALIGN
    assert _crypt(64, d_in=0x1000, d_out=0x1008) == -4  # TDES_ERR_OVERLAP
    assert _crypt(8, d_in=0, d_out=0x1000) == -1  # NULL buffer
    assert _crypt(8, dir=2) == -1
    assert _crypt(8, kernel=7) == -1
    assert _crypt(8, sched=False) == -1
    assert b"overlap" in _crypt_msg(64, 0x1000, 0x1008)
    assert _crypt(0, d_in=0, d_out=0) == 0        # empty: no-op
    assert T.lib().tdes_key_schedule(None, None) == -1
    lib = T.lib()
    assert lib.tdes_probe_valu(9, ctypes.c_void_p(0x1000), 1, 1, None) == -1
    assert lib.tdes_probe_valu(0, None, 1, 1, None) == -1
    assert lib.tdes_probe_copy(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 24, None) == -1
    assert lib.tdes_probe_copy(ctypes.c_void_p(0x1008), ctypes.c_void_p(0x2000), 32, None) == -1


def _host(nbytes=64, h_in=0x1000, h_out=0x10000, d_work=0x100000, work=1 << 20, chunk=1 << 16,
          dir=0, sched=True):
    s = T.key_schedule(bytes(24))
    return T.lib().tdes_ecb_host(ctypes.byref(s) if sched else None, dir, ctypes.c_void_p(h_in),
                                 ctypes.c_void_p(h_out), nbytes, ctypes.c_void_p(d_work), work,
                                 chunk)


def test_host_path_argument_errors():
    # tdes_ecb_host (staged mode: a workspace is given) rejects each of these
    # before any HIP call
    assert _host(sched=False) == -1
    assert _host(dir=2) == -1
    assert _host(chunk=0) == -1
    assert _host(chunk=12) == -2                   # TDES_ERR_LENGTH
    assert _host(nbytes=12) == -2
    assert _host(h_in=0x1004) == -3                # TDES_ERR_ALIGN
    assert _host(d_work=0x100008) == -3            # workspace not 256-byte aligned
    assert _host(h_out=0x1008) == -4               # TDES_ERR_OVERLAP
    assert _host(work=1 << 15) == -1               # workspace smaller than a chunk
    assert b"smaller than one chunk" in T.lib().tdes_last_error()
    assert _host(h_in=0) == -1
    assert _host(nbytes=0, h_in=0, h_out=0, d_work=0) == 0  # empty: no-op


def test_ctr_argument_errors():
    s = T.key_schedule(bytes(24))
    lib = T.lib()
    iv = (ctypes.c_uint8 * 8)()

    def call(nbytes=64, a=0x1000, b=0x100000, ivp=iv, sched=True):
        return lib.tdes_ctr_crypt(ctypes.byref(s) if sched else None, ivp, ctypes.c_void_p(a),
                                  ctypes.c_void_p(b), nbytes, None)
    assert call(ivp=None) == -1
    assert call(sched=False) == -1
    assert call(nbytes=12) == -2
    assert call(a=0x1004) == -3
    assert call(b=0x1008) == -4
    assert call(nbytes=0, a=0, b=0) == 0


def test_cbc_argument_errors():
    s = T.key_schedule(bytes(24))
    lib = T.lib()
    iv = (ctypes.c_uint8 * 8)()

    def call(nbytes=64, a=0x1000, b=0x100000, ivp=iv, sched=True):
        return lib.tdes_cbc_decrypt(ctypes.byref(s) if sched else None, ivp, ctypes.c_void_p(a),
                                    ctypes.c_void_p(b), nbytes, None)
    assert call(ivp=None) == -1
    assert call(sched=False) == -1
    assert call(nbytes=12) == -2
    assert call(a=0x1004) == -3
    assert call(b=0x1008) == -4
    assert call(b=0x1000) == -4  # in place: the ciphertext is re-read
    assert call(nbytes=0, a=0, b=0) == 0


def test_batch_autotune_argument_errors():
    lib = T.lib()
    m = T.BatchConfig()
    a = ctypes.c_void_p(0x1000)

    def call(n=4, reps=2, out=ctypes.byref(m), ws=0x1000, ws_bytes=1 << 20, msgs=0x1000,
             d_in=0x100000, in_bytes=4096, d_out=0x200000, out_bytes=4096):
        return lib.tdes_batch_autotune(ctypes.c_void_p(msgs), n, a, 1, ctypes.c_void_p(d_in),
                                       in_bytes, ctypes.c_void_p(d_out), out_bytes,
                                       ctypes.c_void_p(ws), ws_bytes, None, reps, out)
    assert call(reps=0) == -1
    assert call(out=None) == -1
    assert call(n=0) == -1
    assert call(ws_bytes=8) == -1       # workspace too small
    assert call(ws=0x1004) == -3        # misaligned
    assert call(msgs=0) == -1
    # the trials rewrite the output from the input: aliasing is refused
    assert call(d_out=0x100000) == -4   # in place
    assert b"must not overlap" in lib.tdes_last_error()
    assert call(d_out=0x100800) == -4   # partial overlap
    assert call(d_in=0x200800) == -4    # output range covers the input's start


def test_auto_kernel_query_needs_a_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present: the GPU tests cover the query")
    assert T.lib().tdes_ecb_auto_kernel(8) == -6
    assert b"no device" in T.lib().tdes_last_error()


def test_batch_autotune_streams_argument_errors():
    lib = T.lib()
    m = T.BatchConfig()
    a = ctypes.c_void_p(0x1000)

    def arr(*v):
        return (ctypes.c_void_p * len(v))(*[ctypes.c_void_p(x) for x in v])

    def call(outs=(0x200000, 0x300000), wss=(0x1000, 0x400000), n=2, null=None, d_in=0x100000):
        o = None if null == "outs" else arr(*outs)
        w = None if null == "wss" else arr(*wss)
        st = None if null == "streams" else arr(*([0] * max(1, n)))
        return lib.tdes_batch_autotune_streams(a, 4, a, 1, ctypes.c_void_p(d_in), 4096, o, 4096,
                                               w, 1 << 16, st, n, 2, ctypes.byref(m))
    assert call(n=0) == -1
    assert call(n=9, outs=[0x200000 + 0x2000 * i for i in range(9)],
                wss=[0x1000000 + 0x20000 * i for i in range(9)]) == -1
    for what in ("outs", "wss", "streams"):
        assert call(null=what) == -1, what
    assert call(outs=(0x200000, 0x200800)) == -4      # the lanes' outputs overlap
    assert b"outputs overlap" in lib.tdes_last_error()
    assert call(wss=(0x1000, 0x8000)) == -4            # the lanes' workspaces overlap
    assert b"workspaces overlap" in lib.tdes_last_error()
    assert call(outs=(0x200000, 0x100000)) == -4       # a lane writes over the input
    assert call(wss=(0x1000, 0x400004)) == -3          # misaligned workspace


def test_batch_submit_argument_errors():
    lib = T.lib()
    a = ctypes.c_void_p(0x1000)

    def call(n=4, ws=0x1000, ws_bytes=1 << 20, msgs=0x1000, sched=0x1000, n_sched=1, d_in=0x100000):
        return lib.tdes_batch_submit(ctypes.c_void_p(msgs), n, ctypes.c_void_p(sched), n_sched,
                                     ctypes.c_void_p(d_in), 4096, a, 4096, ctypes.c_void_p(ws),
                                     ws_bytes, None)
    assert call(n=0, msgs=0, ws=0) == 0  # empty batch: no-op
    assert call(ws_bytes=8) == -1
    assert b"workspace too small" in lib.tdes_last_error()
    assert call(n_sched=0) == -1
    assert call(n_sched=(1 << 22) + 1) == -1
    assert b"schedules: at most" in lib.tdes_last_error()
    assert call(n=(1 << 31) + 1, ws_bytes=1 << 40) == -1
    assert b"messages: at most" in lib.tdes_last_error()
    assert call(sched=0x1008) == -3     # schedules must be 16-byte aligned
    assert call(d_in=0x100004) == -3
    assert call(msgs=0) == -1


def test_batch_config_cache_file(tmp_path):
    # The tuning cache: entries keyed by architecture name and CU count,
    # written and read back, other entries kept, invalid ones ignored.
    path = str(tmp_path / "sub" / "tune.json")
    assert T.batch_config_load(path, "gfx950:sramecc+:xnack-", 256) is None  # no file
    T.batch_config_save(path, "gfx950:sramecc+:xnack-", 256, 4, 4, 3, 201.5)
    T.batch_config_save(path, "gfx950:sramecc+:xnack-", 128, 16, 3, 1, 99.0)
    T.batch_config_save(path, "gfx942:sramecc+:xnack-", 304, 8, 4, 2)
    got = T.batch_config_load(path, "gfx950:sramecc+:xnack-", 256)
    assert (got["kmax"], got["waves"], got["grid_mult"]) == (4, 4, 3)
    got = T.batch_config_load(path, "gfx950:sramecc+:xnack-", 128)
    assert (got["kmax"], got["waves"], got["grid_mult"]) == (16, 3, 1)
    assert T.batch_config_load(path, "gfx950:sramecc+:xnack-", 255) is None  # CU count differs
    assert T.batch_config_load(path, "gfx950", 256) is None                  # name differs
    # replacing an entry keeps the others
    T.batch_config_save(path, "gfx950:sramecc+:xnack-", 256, 8, 3, 4, 180.0)
    got = T.batch_config_load(path, "gfx950:sramecc+:xnack-", 256)
    assert (got["kmax"], got["waves"], got["grid_mult"]) == (8, 3, 4)
    assert T.batch_config_load(path, "gfx942:sramecc+:xnack-", 304)["kmax"] == 8
    text = open(path).read()
    assert text.count('"device"') == 3 and text.startswith('{"format": "tdes-batch-tune-1"')
    import json
    doc = json.loads(text)  # the file is valid JSON
    assert len(doc["entries"]) == 3
    # configurations that are not compiled variants are refused, and ignored
    # when found in a file
    with pytest.raises(T.TdesError):
        T.batch_config_save(path, "gfx950", 256, 5, 4, 2)
    with pytest.raises(T.TdesError):
        T.batch_config_save(path, "gfx950", 256, 8, 4, 9)
    with pytest.raises(T.TdesError):
        T.batch_config_save(path, 'gfx"950', 256, 8, 4, 2)
    with pytest.raises(T.TdesError):
        T.batch_config_save("", "gfx950", 256, 8, 4, 2)
    bad = tmp_path / "bad.json"
    bad.write_text('{"entries": [\n{"device": "gfx950", "cus": 256, "kmax": 5, "waves": 4, '
                   '"grid_mult": 2},\n{"device": "gfx950", "cus": 256, "kmax": 8}\n]}\n')
    assert T.batch_config_load(str(bad), "gfx950", 256) is None
    bad.write_text("not json at all\n")
    assert T.batch_config_load(str(bad), "gfx950", 256) is None


def test_batch_config_needs_a_device_or_a_valid_value():
    lib = T.lib()
    c = T.BatchConfig(5, 4, 2, 0)
    assert lib.tdes_batch_set_config(ctypes.byref(c)) == -1   # not a compiled variant
    c = T.BatchConfig(8, 4, 0, 0)
    assert lib.tdes_batch_set_config(ctypes.byref(c)) == -1   # grid multiplier 0
    assert lib.tdes_batch_set_config(None) == -1
    assert lib.tdes_batch_get_config(None) == -1


def _crypt_msg(n, a, b):
    _crypt(n, a, b)
    return T.lib().tdes_last_error()


def test_tables_match_oracle_transcription():
    pairs = {"pc_1": DT.PC1, "shift_keys": DT.SHIFTS, "pc_2": DT.PC2, "initial_perm": DT.IP,
             "exp_d": DT.E, "per": DT.P, "final_perm": DT.FP}
    for name, mine in pairs.items():
        assert oracle.table(name) == list(mine), name
    flat = [v for box in DT.SBOX for row in box for v in row]
    assert oracle.table("s") == flat


def test_sbox_networks_exhaustive():
    nets = load_networks()
    for box in range(8):
        for v in range(64):
            assert evaluate(nets[box], v) == oracle.sbox(box, v), (box, v)


def test_folded_networks_exhaustive():
    # The networks as the kernels run them: a second-use input whose key mask
    # is folded into its gates enters them raw, with the mask as the third
    # operand; every output must be the S-box of (input ^ mask), for all 64
    # inputs and every value of the folded masks.
    nets = load_networks()
    _, folded = emit.plan(nets)
    assert len(folded) == 48 - int(re.search(r"#define BS_XORS_PER_ROUND (\d+)",
                                             E._header("bitslice_gen.h")).group(1))
    for box in range(8):
        f = emit.box_network(nets, box)
        for v in range(64):
            for mbits in range(1 << len(f["folded"])):
                sig = {q: (v >> (5 - q)) & 1 for q in range(6)}
                eff = v
                for i, q in enumerate(f["folded"]):
                    m = (mbits >> i) & 1
                    sig[MASK_BASE + q] = m
                    eff ^= m << (5 - q)
                for i, (a, b, c, imm) in enumerate(f["gates"]):
                    sig[6 + i] = (imm >> ((sig[a] << 2) | (sig[b] << 1) | sig[c])) & 1
                got = 0
                for sg, neg in f["outs"]:
                    got = (got << 1) | (sig[sg] ^ neg)
                assert got == oracle.sbox(box, eff), (box, v, mbits)


def test_generated_headers_are_current():
    assert all(E.generated_headers_match().values()), E.generated_headers_match()


def _kk(key, dec, kernel):
    return T.kernel_key_bytes(T.key_schedule(key), T.DECRYPT if dec else T.ENCRYPT, kernel)


@pytest.mark.parametrize("kind", ["three_key", "two_key", "all_zero", "all_one"])
def test_bitslice_emulation_matches_oracle(kind):
    # all-zero and all-one keys make every key mask 0 or ~0 at once
    g = W.rng(W.SEED_BASE + 0xC00 + (kind == "two_key"))
    key = W.key_bundle(g, two_key=kind == "two_key")
    if kind == "all_zero":
        key = np.zeros(24, np.uint8)
    elif kind == "all_one":
        key = np.full(24, 0xFF, np.uint8)
    data = W.uniform_bytes(g, 8 * 29)  # a partial lane
    ct = E.bitslice_ecb(_kk(key, False, T.KERNEL_BITSLICE), data)
    assert np.array_equal(ct, oracle.tdes_ecb(key, data))
    pt = E.bitslice_ecb(_kk(key, True, T.KERNEL_BITSLICE), ct)
    assert np.array_equal(pt, data)


def test_spbox_emulation_matches_oracle():
    g = W.rng(W.SEED_BASE + 0xC10)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 8 * 6)
    ct = E.spbox_ecb(_kk(key, False, T.KERNEL_SPBOX), data)
    assert np.array_equal(ct, oracle.tdes_ecb(key, data))
    pt = E.spbox_ecb(_kk(key, True, T.KERNEL_SPBOX), ct)
    assert np.array_equal(pt, data)


def test_kernel_key_bytes_errors():
    s = T.key_schedule(bytes(24))
    buf = ctypes.create_string_buffer(16)
    assert T.lib().tdes_kernel_key_bytes(ctypes.byref(s), 0, 1, buf, 16) == -1
    assert T.lib().tdes_kernel_key_bytes(ctypes.byref(s), 3, 1, buf, 16) == -1
