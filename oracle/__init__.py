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
