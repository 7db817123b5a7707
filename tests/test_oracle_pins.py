"""Pins for the oracle's DES / 3DES arithmetic, each against something other
than the oracle itself.

* Exact values: OpenSSL's ``des-ede3`` and legacy ``des-ecb`` ciphers, run as
  a black box on seeded random keys and data (the oracle shares no code with
  it).  This fixes bit order, S-box addressing, rotation schedule and the
  final swap together.
* Structure (Sec. III-B): decryption is the same procedure with reversed
  round keys, so dec(enc(x)) = x only if the halves are recombined as
  R16 || L16; and EDE with K1 = K2 = K3 is single DES.
* Complementation: E bit selection, key mixing by XOR and the XOR into the
  left half give DES(~k, ~p) = ~DES(k, p).
* Weak and semi-weak keys, derived here from the PC-1 table: keys whose two
  28-bit halves are constant (or alternate 0101...) have all-equal (or
  pairwise reversed) round keys, so encryption is an involution (or the
  partner key decrypts).  A wrong rotation schedule or half split breaks
  these.
* Parity bits are never read.
* The paper's worked S-box example (Sec. III-B), stored under tests/golden.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2007_10752_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gen(i):
    return W.rng(W.SEED_BASE + 0x900 + i)


def _openssl(cipher_args, key, data):
    exe = shutil.which("openssl")
    if exe is None:
        pytest.skip("openssl not available")
    r = subprocess.run([exe, "enc"] + cipher_args + ["-nopad", "-K", bytes(key).hex()],
                       input=bytes(data), capture_output=True, timeout=60)
    if r.returncode != 0:
        pytest.skip("openssl refused: %s" % r.stderr.decode(errors="replace")[:200])
    return np.frombuffer(r.stdout, dtype=np.uint8)


def _openssl_dec(cipher_args, key, data):
    return _openssl(cipher_args + ["-d"], key, data)


@pytest.mark.parametrize("case", range(6))
def test_tdes_matches_openssl(case):
    g = _gen(case)
    key = W.key_bundle(g, two_key=(case % 3 == 2))
    data = W.uniform_bytes(g, 8 * 257)
    ct = oracle.tdes_ecb(key, data)
    assert np.array_equal(ct, _openssl(["-des-ede3"], key, data))
    pt = oracle.tdes_ecb(key, data, decrypt=True)
    assert np.array_equal(pt, _openssl_dec(["-des-ede3"], key, data))


@pytest.mark.parametrize("case", range(3))
def test_des_matches_openssl(case):
    g = _gen(100 + case)
    key = W.key_bundle(g)[:8]
    data = W.uniform_bytes(g, 8 * 129)
    args = ["-des-ecb", "-provider", "legacy", "-provider", "default"]
    assert np.array_equal(oracle.des_ecb(key, data), _openssl(args, key, data))
    assert np.array_equal(oracle.des_ecb(key, data, True), _openssl_dec(args, key, data))


# ---- CTR and CBC (the oracle's other modes) ----------------------------------

def _iv_cases(g):
    # a random IV, and one three blocks below 2^64 so the counter wraps
    return [W.uniform_bytes(g, 8), np.frombuffer(((1 << 64) - 3).to_bytes(8, "big"), np.uint8)]


def test_ctr_matches_openssl_ecb_of_counter_blocks():
    # Counter blocks built here with Python integers, encrypted by OpenSSL
    # as a black box, XORed with the data.
    g = _gen(600)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 8 * 77)
    for iv in _iv_cases(g):
        v = int.from_bytes(bytes(iv), "big")
        counters = b"".join(((v + i) % (1 << 64)).to_bytes(8, "big") for i in range(77))
        ks = _openssl(["-des-ede3"], key, np.frombuffer(counters, np.uint8))
        assert np.array_equal(oracle.tdes_ctr(key, iv, data), data ^ ks)


def test_ctr_is_its_own_inverse_and_zero_data_gives_keystream():
    g = _gen(601)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 8 * 50)
    iv = W.uniform_bytes(g, 8)
    ct = oracle.tdes_ctr(key, iv, data)
    assert np.array_equal(oracle.tdes_ctr(key, iv, ct), data)
    zero = oracle.tdes_ctr(key, iv, np.zeros(16, np.uint8))
    assert np.array_equal(zero[:8], oracle.tdes_ecb(key, iv))


@pytest.mark.parametrize("case", range(3))
def test_cbc_matches_openssl(case):
    g = _gen(610 + case)
    key = W.key_bundle(g, two_key=case == 2)
    data = W.uniform_bytes(g, 8 * 93)
    iv = W.uniform_bytes(g, 8)
    args = ["-des-ede3-cbc", "-iv", bytes(iv).hex()]
    ct = oracle.tdes_cbc_encrypt(key, iv, data)
    assert np.array_equal(ct, _openssl(args, key, data))
    assert np.array_equal(oracle.tdes_cbc_decrypt(key, iv, data), _openssl_dec(args, key, data))
    assert np.array_equal(oracle.tdes_cbc_decrypt(key, iv, ct), data)


@pytest.mark.parametrize("two_key", [False, True])
def test_decrypt_inverts_encrypt(two_key):
    g = _gen(200 + two_key)
    key = W.key_bundle(g, two_key=two_key)
    data = W.uniform_bytes(g, 8 * 300)
    assert np.array_equal(oracle.tdes_ecb(key, oracle.tdes_ecb(key, data), True), data)
    assert np.array_equal(oracle.tdes_ecb(key, oracle.tdes_ecb(key, data, True)), data)
    k1 = key[:8]
    assert np.array_equal(oracle.des_ecb(k1, oracle.des_ecb(k1, data), True), data)


def test_equal_keys_give_single_des():
    # Sec. III-B: with all three base keys equal the system behaves like DES.
    g = _gen(300)
    k = W.key_bundle(g)[:8]
    key = np.concatenate([k, k, k])
    data = W.uniform_bytes(g, 8 * 200)
    assert np.array_equal(oracle.tdes_ecb(key, data), oracle.des_ecb(k, data))
    assert np.array_equal(oracle.tdes_ecb(key, data, True), oracle.des_ecb(k, data, True))


def test_ede_order_is_not_ded():
    # E_K3(D_K2(E_K1(p))): compose single DES calls in the paper's order.
    g = _gen(301)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 8 * 64)
    k1, k2, k3 = key[:8], key[8:16], key[16:]
    ede = oracle.des_ecb(k3, oracle.des_ecb(k2, oracle.des_ecb(k1, data), True))
    assert np.array_equal(oracle.tdes_ecb(key, data), ede)
    ded = oracle.des_ecb(k1, oracle.des_ecb(k2, oracle.des_ecb(k3, data, True)), True)
    assert np.array_equal(oracle.tdes_ecb(key, data, True), ded)


def test_complementation():
    g = _gen(400)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 8 * 128)
    for dec in (False, True):
        a = oracle.tdes_ecb(key, data, dec)
        b = oracle.tdes_ecb(~key, ~data, dec)
        assert np.array_equal(b, ~a)
        a1 = oracle.des_ecb(key[:8], data, dec)
        assert np.array_equal(oracle.des_ecb(~key[:8], ~data, dec), ~a1)


def test_parity_bits_are_ignored():
    g = _gen(500)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 8 * 64)
    ref = oracle.tdes_ecb(key, data)
    for byte in range(24):
        k = key.copy()
        k[byte] ^= 1  # DES bit 8 of this byte
        assert np.array_equal(oracle.tdes_ecb(k, data), ref)
    k = key ^ np.uint8(1)
    assert np.array_equal(oracle.tdes_ecb(k, data, True), oracle.tdes_ecb(key, data, True))


def _key_from_halves(c_bits, d_bits, fill=0):
    """64-bit key whose PC-1 image has C = c_bits, D = d_bits (28 each)."""
    pc1 = oracle.table("pc_1")
    bits = [fill] * 65
    for j in range(28):
        bits[pc1[j]] = c_bits[j]
        bits[pc1[28 + j]] = d_bits[j]
    key = np.zeros(8, dtype=np.uint8)
    for i in range(8):
        v = 0
        for j in range(8):
            v = 2 * v + bits[8 * i + j + 1]
        key[i] = v
    return key


ZERO, ONE = [0] * 28, [1] * 28
ALT01, ALT10 = [j % 2 for j in range(28)], [(j + 1) % 2 for j in range(28)]


@pytest.mark.parametrize("c,d", [(ZERO, ZERO), (ZERO, ONE), (ONE, ZERO), (ONE, ONE)])
def test_weak_keys_are_involutions(c, d):
    key = _key_from_halves(c, d)
    sub = oracle.key_schedule(key)
    assert len(set(sub)) == 1
    data = W.uniform_bytes(_gen(600), 8 * 64)
    assert np.array_equal(oracle.des_ecb(key, oracle.des_ecb(key, data)), data)


def _swap_alt(h):
    return ALT10 if h is ALT01 else ALT01 if h is ALT10 else h


@pytest.mark.parametrize("c,d", [(ALT01, ZERO), (ALT01, ONE), (ZERO, ALT01), (ONE, ALT01),
                                 (ALT01, ALT01), (ALT01, ALT10)])
def test_semi_weak_pairs(c, d):
    k1 = _key_from_halves(c, d)
    k2 = _key_from_halves(_swap_alt(c), _swap_alt(d))
    s1, s2 = oracle.key_schedule(k1), oracle.key_schedule(k2)
    assert s2 == s1[::-1]
    data = W.uniform_bytes(_gen(700), 8 * 64)
    assert np.array_equal(oracle.des_ecb(k2, oracle.des_ecb(k1, data)), data)
    assert np.array_equal(oracle.des_ecb(k1, oracle.des_ecb(k2, data)), data)


def test_paper_sbox_worked_example():
    rows = {}
    boxes = {}
    with open(os.path.join(GOLDEN, "sbox_worked_example.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "box":
                boxes[int(line[1])] = int(line[2])
            else:
                rows[line[0]] = line[1]
    six = int(rows["six_bits"], 2)
    assert (six >> 1) & 0xF == int(rows["col_index"])
    assert ((six >> 5) << 1 | (six & 1)) == int(rows["row_index"])
    for box, val in boxes.items():
        assert oracle.sbox(box - 1, six) == val


def test_empty_and_single_block():
    key = W.key_bundle(_gen(800))
    assert oracle.tdes_ecb(key, np.zeros(0, np.uint8)).size == 0
    one = W.uniform_bytes(_gen(801), 8)
    assert np.array_equal(oracle.tdes_ecb(key, oracle.tdes_ecb(key, one), True), one)


def test_rejects_partial_block():
    with pytest.raises(ValueError):
        oracle.tdes_ecb(bytes(24), np.zeros(12, np.uint8))
