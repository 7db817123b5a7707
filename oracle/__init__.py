"""Oracle for DES / Triple-DES EDE over independent 64-bit blocks (ECB).

TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
CPU-baseline leg of the benchmark to check the GPU library.  The library does
not import, load or call anything here, and nothing here comes from it.

A thin ctypes wrapper over ``tdes_oracle.c`` (plain, bit-at-a-time C; one
unsigned char per bit as in the paper's memory design, Sec. IV-C).  Keys and
data are bytes-like or numpy uint8 arrays; DES bit 1 is the most significant
bit of byte 0.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.OUT
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build()
    lib = ctypes.CDLL(path)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.oracle_key_schedule.argtypes = [u8p, ctypes.POINTER(ctypes.c_uint64)]
    lib.oracle_key_schedule.restype = None
    lib.oracle_sbox.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.oracle_sbox.restype = ctypes.c_int
    for name in ("oracle_des_ecb", "oracle_tdes_ecb"):
        fn = getattr(lib, name)
        fn.argtypes = [u8p, u8p, u8p, ctypes.c_size_t, ctypes.c_int]
        fn.restype = None
    lib.oracle_table.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
    lib.oracle_table.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _u8(buf, n=None):
    a = np.ascontiguousarray(np.frombuffer(bytes(buf), dtype=np.uint8)
                             if isinstance(buf, (bytes, bytearray)) else buf, dtype=np.uint8)
    if n is not None and a.size != n:
        raise ValueError("expected %d bytes, got %d" % (n, a.size))
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def key_schedule(key8):
    """16 round keys of one 64-bit key (Sec. III-A), as ints; bit 1 of a
    round key is bit 47 of the int."""
    k = _u8(key8, 8)
    out = (ctypes.c_uint64 * 16)()
    _load().oracle_key_schedule(_ptr(k), out)
    return [int(v) for v in out]


def sbox(box, six_bits):
    """Value of S-box ``box`` (0..7) for the 6-bit input b1..b6 (b1 = bit 5)."""
    return int(_load().oracle_sbox(int(box), int(six_bits)))


def _ecb(fn, key, nkey, data, decrypt):
    k = _u8(key, nkey)
    d = _u8(data).reshape(-1)
    if d.size % 8:
        raise ValueError("length %d is not a multiple of 8 bytes" % d.size)
    out = np.empty_like(d)
    fn(_ptr(k), _ptr(d), _ptr(out), d.size, 1 if decrypt else 0)
    return out


def des_ecb(key8, data, decrypt=False):
    """Single DES, ECB (Sec. III-B)."""
    return _ecb(_load().oracle_des_ecb, key8, 8, data, decrypt)


def tdes_ecb(key24, data, decrypt=False):
    """Triple-DES EDE, ECB, key bundle K1||K2||K3 (Sec. III-B equations)."""
    return _ecb(_load().oracle_tdes_ecb, key24, 24, data, decrypt)


# ---- Other modes over the same block cipher ----------------------------------
# The paper applies 3DES in ECB only (Sec. V).  The modes below are the
# standard ones (NIST SP 800-38A) built on the block cipher above, written
# from their definitions: CTR in Sec. 6.5, CBC in Sec. 6.2.


def tdes_ctr(key24, iv8, data):
    """CTR mode: output block i = input block i XOR E(T_i), with counter
    block T_i = (IV + i) mod 2^64, the whole 64-bit block read as a
    big-endian integer (SP 800-38A Sec. 6.5 and its Appendix B incrementing
    function with m = 64).  Encryption and decryption are the same."""
    d = _u8(data).reshape(-1)
    if d.size % 8:
        raise ValueError("length %d is not a multiple of 8 bytes" % d.size)
    iv = int.from_bytes(bytes(_u8(iv8, 8)), "big")
    n = d.size // 8
    counters = (np.uint64(iv) + np.arange(n, dtype=np.uint64))  # wraps mod 2^64
    blocks = counters.astype(">u8").view(np.uint8)
    return d ^ tdes_ecb(key24, blocks)


def tdes_cbc_encrypt(key24, iv8, data):
    """CBC encryption (SP 800-38A Sec. 6.2): C_i = E(P_i XOR C_{i-1}), with
    C_{-1} = IV; one block after another."""
    d = _u8(data).reshape(-1, 8)
    out = np.empty_like(d)
    prev = _u8(iv8, 8)
    for i in range(d.shape[0]):
        prev = tdes_ecb(key24, d[i] ^ prev)
        out[i] = prev
    return out.reshape(-1)


def tdes_cbc_decrypt(key24, iv8, data):
    """CBC decryption (SP 800-38A Sec. 6.2): P_i = D(C_i) XOR C_{i-1}, with
    C_{-1} = IV; every block independent of the others' results."""
    d = _u8(data).reshape(-1)
    if d.size % 8:
        raise ValueError("length %d is not a multiple of 8 bytes" % d.size)
    prev = np.concatenate([_u8(iv8, 8), d[:-8]]) if d.size else d
    return tdes_ecb(key24, d, decrypt=True) ^ prev


TABLES = ("pc_1", "shift_keys", "pc_2", "initial_perm", "exp_d", "s", "per", "final_perm")


def table(name):
    """The oracle's own transcription of an Appendix A array, as a list
    (``s`` is flattened box-major: s[box][row][col])."""
    buf = (ctypes.c_int * 512)()
    n = _load().oracle_table(TABLES.index(name), buf, 512)
    return list(buf[:n])


def set_threads(n):
    """Set the OpenMP thread count (n <= 0 leaves it); returns the count in use."""
    return int(_load().oracle_set_threads(int(n)))
