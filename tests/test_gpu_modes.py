"""GPU parity of the other modes over the bitsliced kernel, bit for bit
against the oracle: CTR (tdes_ctr_crypt) and CBC decryption
(tdes_cbc_decrypt).

The cases are:

* ragged sizes around the 16 KiB wave chunk and the 32-block lane slice;
* counters whose low word carries into the high word, and counters that
  wrap past 2^64;
* 8-byte-aligned and in-place buffers;
* the 64 MiB case in full;
* the 1 GiB case on seeded runs of blocks, checked one run at a time (the
  oracle's CTR from the IV advanced to the run's first block).

CBC decryption: the same ragged sizes (the first block of every wave chunk
takes its previous block from the chunk before, the buffer's first block
the IV), 8-byte-aligned buffers, the 64 MiB case in full, and the 1 GiB
case on seeded runs (the oracle's CBC decryption of a run, with the
ciphertext block before the run as its IV)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2007_10752_amd import tdes as T
from paper_2007_10752_amd import workloads as W

pytestmark = pytest.mark.gpu

RAGGED = [1, 2, 31, 32, 33, 2047, 2048, 2049, 4097, 3 * 2048 + 5, 12345]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _iv(v):
    return np.frombuffer((v % (1 << 64)).to_bytes(8, "big"), np.uint8).copy()


def _ctr_gpu(torch, key, iv, data, offset=0, inplace=False):
    buf = torch.zeros(data.size + offset, dtype=torch.uint8, device="cuda")
    x = buf[offset:]
    x.copy_(torch.from_numpy(data))
    out = x if inplace else torch.empty_like(x)
    T.ctr(key, iv, x, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("nblocks", RAGGED)
def test_ctr_ragged_sizes(torch_dev, nblocks):
    g = W.rng(W.SEED_BASE + 0x700 + nblocks)
    key = W.key_bundle(g)
    iv = W.uniform_bytes(g, 8)
    data = W.uniform_bytes(g, 8 * nblocks)
    _say("ctr ragged", nblocks)
    got = _ctr_gpu(torch_dev, key, iv, data)
    assert np.array_equal(got, oracle.tdes_ctr(key, iv, data))
    # its own inverse
    assert np.array_equal(_ctr_gpu(torch_dev, key, iv, got), data)


@pytest.mark.parametrize("start", [(1 << 32) - 100, (1 << 64) - 3000, (1 << 64) - 1, 0])
def test_ctr_counter_carries_and_wraps(torch_dev, start):
    g = W.rng(W.SEED_BASE + 0x710)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 8 * 6000)
    iv = _iv(start)
    _say("ctr counter start", hex(start))
    got = _ctr_gpu(torch_dev, key, iv, data)
    assert np.array_equal(got, oracle.tdes_ctr(key, iv, data))


@pytest.mark.parametrize("offset,inplace", [(8, False), (0, True), (8, True)])
def test_ctr_unaligned_and_in_place(torch_dev, offset, inplace):
    g = W.rng(W.SEED_BASE + 0x720 + offset + inplace)
    key = W.key_bundle(g)
    iv = W.uniform_bytes(g, 8)
    data = W.uniform_bytes(g, 3 * 16384 + 8 * 37)
    _say("ctr offset", offset, "inplace", inplace)
    got = _ctr_gpu(torch_dev, key, iv, data, offset=offset, inplace=inplace)
    assert np.array_equal(got, oracle.tdes_ctr(key, iv, data))


def test_ctr_64mib_full(torch_dev):
    g = W.rng(W.SEED_BASE + 1)
    data = W.uniform_bytes(g, 8 * 8388608)
    key = W.key_bundle(W.rng(W.SEED_BASE + 1 + W.KEY_SEED_OFFSET), two_key=True)
    iv = _iv((1 << 64) - 4096)  # wraps early in the buffer
    _say("ctr 64MiB")
    got = _ctr_gpu(torch_dev, key, iv, data)
    assert np.array_equal(got, oracle.tdes_ctr(key, iv, data))


def test_ctr_1gib_runs(torch_dev):
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 2)
    key = W.key_bundle(W.rng(W.SEED_BASE + 2 + W.KEY_SEED_OFFSET))
    iv_v = int.from_bytes(bytes(W.uniform_bytes(g, 8)), "big")
    _say("ctr 1GiB")
    x = torch.from_numpy(W.uniform_bytes(g, 1 << 30)).cuda()
    out = torch.empty_like(x)
    T.ctr(key, _iv(iv_v), x, out)
    torch.cuda.synchronize()
    nblk = (1 << 30) // 8
    run = 512
    starts = np.sort(W.rng(W.SEED_BASE + 0x730).choice(nblk // run, 64, replace=False)) * run
    starts = np.concatenate([[0], starts, [nblk - run]])
    for s0 in starts.tolist():
        a, b = 8 * s0, 8 * (s0 + run)
        want = oracle.tdes_ctr(key, _iv(iv_v + s0), x[a:b].cpu().numpy())
        assert np.array_equal(out[a:b].cpu().numpy(), want), s0


def _cbc_gpu(torch, key, iv, data, offset=0):
    buf = torch.zeros(data.size + offset, dtype=torch.uint8, device="cuda")
    x = buf[offset:]
    x.copy_(torch.from_numpy(data))
    out = T.cbc_decrypt(key, iv, x)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("nblocks", RAGGED)
def test_cbc_decrypt_ragged_sizes(torch_dev, nblocks):
    g = W.rng(W.SEED_BASE + 0x740 + nblocks)
    key = W.key_bundle(g)
    iv = W.uniform_bytes(g, 8)
    data = W.uniform_bytes(g, 8 * nblocks)
    _say("cbc ragged", nblocks)
    got = _cbc_gpu(torch_dev, key, iv, data)
    assert np.array_equal(got, oracle.tdes_cbc_decrypt(key, iv, data))


def test_cbc_decrypt_round_trip_and_unaligned(torch_dev):
    g = W.rng(W.SEED_BASE + 0x750)
    key = W.key_bundle(g, two_key=True)
    iv = W.uniform_bytes(g, 8)
    plain = W.uniform_bytes(g, 8 * 3000)
    ct = oracle.tdes_cbc_encrypt(key, iv, plain)
    _say("cbc round trip")
    assert np.array_equal(_cbc_gpu(torch_dev, key, iv, ct), plain)
    assert np.array_equal(_cbc_gpu(torch_dev, key, iv, ct, offset=8), plain)


def test_cbc_decrypt_refuses_in_place(torch_dev):
    torch = torch_dev
    x = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(T.TdesError) as e:
        T.cbc_decrypt(bytes(24), bytes(8), x, x)
    assert e.value.status == -4


def test_cbc_decrypt_64mib_full(torch_dev):
    g = W.rng(W.SEED_BASE + 1)
    data = W.uniform_bytes(g, 8 * 8388608)
    key = W.key_bundle(W.rng(W.SEED_BASE + 1 + W.KEY_SEED_OFFSET))
    iv = W.uniform_bytes(W.rng(W.SEED_BASE + 0x760), 8)
    _say("cbc 64MiB")
    got = _cbc_gpu(torch_dev, key, iv, data)
    assert np.array_equal(got, oracle.tdes_cbc_decrypt(key, iv, data))


def test_cbc_decrypt_1gib_runs(torch_dev):
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 2)
    key = W.key_bundle(W.rng(W.SEED_BASE + 2 + W.KEY_SEED_OFFSET))
    iv = W.uniform_bytes(g, 8)
    _say("cbc 1GiB")
    x = torch.from_numpy(W.uniform_bytes(g, 1 << 30)).cuda()
    out = T.cbc_decrypt(key, iv, x)
    torch.cuda.synchronize()
    nblk = (1 << 30) // 8
    run = 512
    starts = np.sort(W.rng(W.SEED_BASE + 0x770).choice(nblk // run, 64, replace=False)) * run
    starts = np.concatenate([[0], starts, [nblk - run]])
    for s0 in starts.tolist():
        a, b = 8 * s0, 8 * (s0 + run)
        run_iv = iv if s0 == 0 else x[a - 8:a].cpu().numpy()
        want = oracle.tdes_cbc_decrypt(key, run_iv, x[a:b].cpu().numpy())
        assert np.array_equal(out[a:b].cpu().numpy(), want), s0
