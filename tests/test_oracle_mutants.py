"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a private copy of the oracle's C source
(a dropped term, a transposed index, a wrong order or convention), builds it
on the CPU and checks that the pins used in test_oracle_pins.py (OpenSSL
black-box values, dec(enc(x)) = x) reject it.  Nothing here touches the GPU.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle import build as obuild
from paper_2007_10752_amd import workloads as W

MUTANTS = {
    "combine_L16_R16": ("pre[j] = right[j];\n        pre[32 + j] = left[j];",
                        "pre[j] = left[j];\n        pre[32 + j] = right[j];"),
    "sbox_row_bits_swapped": ("int row = 2 * six[0] + six[5];", "int row = 2 * six[5] + six[0];"),
    "sbox_col_reversed": ("int col = 8 * six[1] + 4 * six[2] + 2 * six[3] + six[4];",
                          "int col = six[1] + 2 * six[2] + 4 * six[3] + 8 * six[4];"),
    "sbox_output_lsb_first": ("sub[4 * b + q + 1] = (v >> (3 - q)) & 1;",
                              "sub[4 * b + q + 1] = (v >> q) & 1;"),
    "rotation_amounts_all_one": ("rotate_left_28(c, shift_keys[i]);", "rotate_left_28(c, 1);"),
    "rotation_table_reversed": ("rotate_left_28(d, shift_keys[i]);",
                                "rotate_left_28(d, shift_keys[15 - i]);"),
    "input_bits_lsb_first": ("bits[8 * i + j + 1] = (bytes[i] >> (7 - j)) & 1;",
                             "bits[8 * i + j + 1] = (bytes[i] >> j) & 1;"),
    "ip_as_scatter": ("permute(t, in, initial_perm, 64);", "permute(t, in, final_perm, 64);"),
    "dropped_key_bit": ("x[j] = e[j] ^ k[j];", "x[j] = e[j] ^ (j == 7 ? 0 : k[j]);"),
    "decrypt_key_off_by_one": ("rk->k[decrypt ? 15 - round : round]",
                               "rk->k[decrypt ? (16 - round) % 16 : round]"),
    "ded_instead_of_ede": ("des_bits(a, c, &rk1, 0);\n            des_bits(c, a, &rk2, 1);\n            des_bits(a, c, &rk3, 0);",
                           "des_bits(a, c, &rk1, 1);\n            des_bits(c, a, &rk2, 0);\n            des_bits(a, c, &rk3, 1);"),
    "sbox5_entries_swapped": ("{14, 11, 2, 12, 4, 7, 13, 1, 5, 0, 15, 10, 3, 9, 8, 6}",
                              "{14, 11, 2, 12, 4, 7, 13, 1, 5, 0, 10, 15, 3, 9, 8, 6}"),
    "expansion_entry": ("28, 29, 28, 29, 30, 31, 32, 1};", "28, 29, 28, 29, 30, 31, 31, 1};"),
}


def _openssl(args, key, data):
    exe = shutil.which("openssl")
    r = subprocess.run([exe, "enc"] + args + ["-nopad", "-K", bytes(key).hex()],
                       input=bytes(data), capture_output=True, timeout=60)
    assert r.returncode == 0
    return np.frombuffer(r.stdout, dtype=np.uint8)


def _build_mutant(tmp_path, name):
    src = open(obuild.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, "mutation site for %s not found exactly once" % name
    path = tmp_path / ("%s.c" % name)
    path.write_text(src.replace(old, new))
    so = tmp_path / ("lib%s.so" % name)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(path)],
                   check=True)
    lib = ctypes.CDLL(str(so))
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.oracle_tdes_ecb.argtypes = [u8p, u8p, u8p, ctypes.c_size_t, ctypes.c_int]
    return lib


def _run(lib, key, data, dec):
    out = np.empty_like(data)
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    lib.oracle_tdes_ecb(p(key), p(data), p(out), data.size, int(dec))
    return out


def _pins_pass(lib):
    g = W.rng(W.SEED_BASE + 0xA00)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 8 * 64)
    ct = _run(lib, key, data, False)
    if not np.array_equal(_run(lib, key, ct, True), data):
        return False
    if shutil.which("openssl") is not None:
        if not np.array_equal(ct, _openssl(["-des-ede3"], key, data)):
            return False
    return True


def test_unmutated_copy_passes(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(obuild.SRC).read()
    path = tmp_path / "plain.c"
    path.write_text(src)
    so = tmp_path / "libplain.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(path)], check=True)
    lib = ctypes.CDLL(str(so))
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.oracle_tdes_ecb.argtypes = [u8p, u8p, u8p, ctypes.c_size_t, ctypes.c_int]
    assert _pins_pass(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    if shutil.which("gcc") is None or shutil.which("openssl") is None:
        pytest.skip("gcc and openssl needed")
    assert not _pins_pass(_build_mutant(tmp_path, name))
