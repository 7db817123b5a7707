"""GPU parity: both HIP kernels, called through the C ABI, against the
oracle, bit for bit (3DES is a deterministic function: one right answer).

Sizes: the 32 KiB case (encrypt then decrypt), ragged sizes around the
16 KiB wave chunk and the 32-block lane slice, unaligned and in-place
buffers, the 64 MiB case in full for 3-key and 2-key bundles in both
directions, and the 1 GiB headline case in the launch configuration the
benchmark times: the whole output against the SHA-256 of the oracle's output
on the same seeded input (tests/golden, written by a script that calls only
the oracle), seeded random positions checked one by one against the oracle,
plus all-zero and repeating-pattern inputs whose every output block must
equal the oracle's output on the one distinct input block.  Also: key
bundles at the edges of the key material, a caller-named stream, a buffer
past 4 GiB (64-bit addressing), and the paper's one-thread-per-bit design
(comparison kernel) against the oracle and the bitsliced kernel.
"""
import hashlib
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2007_10752_amd import tdes as T
from paper_2007_10752_amd import workloads as W

pytestmark = pytest.mark.gpu

KERNELS = ["bitslice", "spbox"]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _to_dev(torch, host, extra=0, offset=0):
    """Device copy of host bytes at a given byte offset inside a bigger
    allocation (offset 8 gives an 8- but not 16-byte aligned pointer)."""
    buf = torch.zeros(host.size + extra + offset, dtype=torch.uint8, device="cuda")
    view = buf[offset: offset + host.size]
    view.copy_(torch.from_numpy(host))
    return buf, view


def _gpu(torch, key, host, decrypt=False, kernel="bitslice", offset=0, inplace=False):
    _, x = _to_dev(torch, host, offset=offset)
    if inplace:
        out = x
    else:
        _, out = _to_dev(torch, np.zeros_like(host), offset=offset)
    T.ecb(key, x, out, decrypt=decrypt, kernel=kernel)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("kernel", KERNELS)
def test_32kib_encrypt_then_decrypt(torch_dev, kernel):
    g = W.rng(W.SEED_BASE + 0)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 4096 * 8)
    _say("32KiB", kernel)
    ct = _gpu(torch_dev, key, data, kernel=kernel)
    assert np.array_equal(ct, oracle.tdes_ecb(key, data))
    pt = _gpu(torch_dev, key, ct, decrypt=True, kernel=kernel)
    assert np.array_equal(pt, data)


RAGGED = [1, 2, 3, 31, 32, 33, 63, 64, 65, 2047, 2048, 2049, 4095, 4097, 3 * 2048 + 5, 12345]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("nblocks", RAGGED)
def test_ragged_sizes(torch_dev, kernel, nblocks):
    g = W.rng(W.SEED_BASE + 0x10 + nblocks)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, nblocks * 8)
    _say("ragged", kernel, nblocks)
    dec = bool(nblocks % 2)
    got = _gpu(torch_dev, key, data, decrypt=dec, kernel=kernel)
    assert np.array_equal(got, oracle.tdes_ecb(key, data, dec))


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("offset,inplace", [(8, False), (0, True), (8, True)])
def test_unaligned_and_in_place(torch_dev, kernel, offset, inplace):
    g = W.rng(W.SEED_BASE + 0x40 + offset + inplace)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 3 * 16384 + 8 * 37)
    _say("offset", offset, "inplace", inplace, kernel)
    got = _gpu(torch_dev, key, data, kernel=kernel, offset=offset, inplace=inplace)
    assert np.array_equal(got, oracle.tdes_ecb(key, data))


def test_zero_length_is_noop(torch_dev):
    torch = torch_dev
    x = torch.zeros(0, dtype=torch.uint8, device="cuda")
    T.ecb(bytes(24), x, x)
    torch.cuda.synchronize()


_C2_CACHE = {}


def _c2_case(two_key):
    if two_key not in _C2_CACHE:
        g = W.rng(W.SEED_BASE + 1)
        data = W.uniform_bytes(g, 8 * 8388608)
        key = W.key_bundle(W.rng(W.SEED_BASE + 1 + W.KEY_SEED_OFFSET), two_key=two_key)
        _say("oracle 64MiB two_key=%s" % two_key)
        _C2_CACHE[two_key] = (key, data, oracle.tdes_ecb(key, data))
    return _C2_CACHE[two_key]


@pytest.mark.parametrize("two_key", [False, True])
@pytest.mark.parametrize("kernel", KERNELS)
def test_64mib_full(torch_dev, kernel, two_key):
    torch = torch_dev
    key, data, want = _c2_case(two_key)
    _say("64MiB", kernel, "two_key", two_key)
    _, x = _to_dev(torch, data)
    ct = torch.empty_like(x)
    T.encrypt(key, x, ct, kernel=kernel)
    pt = torch.empty_like(x)
    T.decrypt(key, ct, pt, kernel=kernel)
    torch.cuda.synchronize()
    assert np.array_equal(ct.cpu().numpy(), want)
    assert torch.equal(pt, x)
    # decryption of the random data itself, on a seeded sample of blocks
    dec = torch.empty_like(x)
    T.decrypt(key, x, dec, kernel=kernel)
    idx = np.sort(W.rng(W.SEED_BASE + 0x50).choice(data.size // 8, 4096, replace=False))
    rows = dec.view(-1, 8)[torch.from_numpy(idx).cuda()].cpu().numpy().reshape(-1)
    sample = data.reshape(-1, 8)[idx].reshape(-1)
    assert np.array_equal(rows, oracle.tdes_ecb(key, sample, decrypt=True))


# The automatic kernel choice: the table kernel up to 6 MiB on a 256-CU
# device (one block per lane, 1.5 waves of resident workgroups), the
# bitsliced kernel above; sizes on both sides of that point, checked in full.
AUTO_SIZES = [8, 32 << 10, (4 << 20) + 8, (6 << 20) - 8, 6 << 20, (6 << 20) + 8, 8 << 20]


def test_auto_kernel_query(torch_dev):
    # the table kernel up to 1.5 passes of its resident workgroups (2 per CU,
    # 1,024 lanes, one 8-byte block each), the bitsliced kernel above
    cus = torch_dev.cuda.get_device_properties(0).multi_processor_count
    limit = 3 * cus * 1024 * 8
    assert T.auto_kernel(8) == "spbox"
    assert T.auto_kernel(limit) == "spbox"
    assert T.auto_kernel(limit + 8) == "bitslice"
    assert T.auto_kernel(1 << 30) == "bitslice"


@pytest.mark.parametrize("nbytes", AUTO_SIZES)
def test_auto_kernel_choice(torch_dev, nbytes):
    g = W.rng(W.SEED_BASE + 0x57)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, nbytes)
    _say("auto", nbytes)
    ct = _gpu(torch_dev, key, data, kernel="auto")
    assert np.array_equal(ct, oracle.tdes_ecb(key, data))
    assert np.array_equal(_gpu(torch_dev, key, ct, decrypt=True, kernel="auto"), data)


# The table kernel spreads few blocks over the CUs with 64, 128, .. 1,024
# working lanes per workgroup (the fewest whose workgroups fit the CUs once):
# block counts at and just past each switch (CUs x lanes), and one between,
# in full against the oracle, both directions.
@pytest.mark.parametrize("lanes,extra", [(64, 0), (64, 1), (96, 37), (128, 0), (128, 1),
                                         (256, 0), (256, 1), (512, 0), (512, 1)])
def test_table_kernel_spread(torch_dev, lanes, extra):
    cus = torch_dev.cuda.get_device_properties(0).multi_processor_count
    nblk = cus * lanes + extra
    g = W.rng(W.SEED_BASE + 0x5A)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 8 * nblk)
    _say("table spread", nblk)
    ct = _gpu(torch_dev, key, data, kernel="spbox")
    assert np.array_equal(ct, oracle.tdes_ecb(key, data))
    assert np.array_equal(_gpu(torch_dev, key, ct, decrypt=True, kernel="spbox"), data)


# Sizes past the point where a lane takes several blocks of the grid-stride
# loop (the table kernel at most 1,024 workgroups of 1,024 lanes: 2^20 blocks
# per sweep), with remainders that leave lanes four, three, two or one block
# more: checked on the blocks near every multiple of 2^20 and a seeded sample.
STRIDE_CASES = [(3 << 20) + 517, (5 << 20) + 9, (7 << 20) + 3]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("nblk", STRIDE_CASES)
def test_grid_stride_remainders(torch_dev, kernel, nblk):
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x58)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 8 * nblk)
    _say("grid-stride", kernel, nblk)
    x = torch.from_numpy(data).cuda()
    out = torch.empty_like(x)
    T.encrypt(key, x, out, kernel=kernel)
    torch.cuda.synchronize()
    near = [np.arange(max(0, k - 1024), min(nblk, k + 1024)) for k in range(0, nblk + 1, 1 << 20)]
    idx = np.concatenate(near + [np.arange(nblk - 2048, nblk),
                                 W.rng(W.SEED_BASE + 0x59).choice(nblk, 1 << 14, replace=False)])
    idx = np.unique(idx)
    ti = torch.from_numpy(idx).cuda()
    got = out.view(-1, 8)[ti].cpu().numpy().reshape(-1)
    sample = data.reshape(-1, 8)[idx].reshape(-1)
    assert np.array_equal(got, oracle.tdes_ecb(key, sample))


GIB = 1 << 30


def _golden_1gib():
    """Fields of tests/golden/ecb_1gib_digest.txt (written by the oracle)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "ecb_1gib_digest.txt")
    fields = {}
    with open(path) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                fields[k] = v
    return fields


@pytest.mark.parametrize("kernel", KERNELS)
def test_1gib_full_and_structured(torch_dev, kernel):
    # The whole 1 GiB uniform output (134,217,728 blocks) against the SHA-256
    # of the oracle's output on the same seeded input, plus a seeded sample
    # and the first and last wave chunks compared block by block.
    torch = torch_dev
    gold = _golden_1gib()
    g = W.rng(int(gold["data_seed"]))
    key = W.key_bundle(W.rng(int(gold["key_seed"])))
    assert bytes(key).hex() == gold["key24"]
    _say("1GiB uniform", kernel)
    data = W.uniform_bytes(g, GIB)
    assert hashlib.sha256(data.tobytes()).hexdigest() == gold["input_sha256"]
    x = torch.from_numpy(data).cuda()
    del data
    out = torch.empty_like(x)
    T.encrypt(key, x, out, kernel=kernel)
    torch.cuda.synchronize()
    assert hashlib.sha256(out.cpu().numpy().tobytes()).hexdigest() == gold["encrypt_sha256"]
    nblk = GIB // 8
    idx = W.rng(W.SEED_BASE + 0x60).choice(nblk, 1 << 16, replace=False)
    idx = np.concatenate([np.arange(2048), idx, np.arange(nblk - 2048, nblk)])
    ti = torch.from_numpy(idx).cuda()
    got = out.view(-1, 8)[ti].cpu().numpy().reshape(-1)
    sample = x.view(-1, 8)[ti].cpu().numpy().reshape(-1)
    assert np.array_equal(got, oracle.tdes_ecb(key, sample))
    del x
    for name, block in (("zero", np.zeros(8, np.uint8)),
                        ("pattern", np.arange(1, 9, dtype=np.uint8))):
        _say("1GiB", name, kernel)
        x = torch.from_numpy(block).cuda().repeat(nblk)
        T.encrypt(key, x, out, kernel=kernel)
        want = torch.from_numpy(oracle.tdes_ecb(key, block)).cuda()
        same = (out.view(-1, 8) == want.view(1, 8)).all()
        torch.cuda.synchronize()
        assert bool(same), name
        del x


def _weak(pattern):
    return np.frombuffer(bytes.fromhex(pattern), dtype=np.uint8)


# Bundles at the edges of the key material: every key bit zero or one (the
# kernels' key masks all zero / all ones), DES weak keys (E_K is its own
# inverse), K1 = K2 = K3 (single DES) and K1 = K2 (EDE reduces to E_K3).
def _edge_bundles():
    g = W.rng(W.SEED_BASE + 0x70)
    k = [W.key_bundle(g)[:8] for _ in range(3)]
    return {
        "zero": np.zeros(24, np.uint8),
        "ones": np.full(24, 0xFF, np.uint8),
        "weak_01": np.tile(_weak("0101010101010101"), 3),
        "weak_fe": np.tile(_weak("FEFEFEFEFEFEFEFE"), 3),
        "weak_e0": np.tile(_weak("E0E0E0E0F1F1F1F1"), 3),
        "weak_1f": np.tile(_weak("1F1F1F1F0E0E0E0E"), 3),
        "single": np.concatenate([k[0], k[0], k[0]]),
        "k1_eq_k2": np.concatenate([k[0], k[0], k[1]]),
        "two_key": np.concatenate([k[0], k[1], k[0]]),
    }


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name", list(_edge_bundles()))
def test_key_edge_cases(torch_dev, kernel, name):
    key = _edge_bundles()[name]
    data = W.uniform_bytes(W.rng(W.SEED_BASE + 0x71), 8 * 4099)
    _say("key edge", name, kernel)
    for dec in (False, True):
        got = _gpu(torch_dev, key, data, decrypt=dec, kernel=kernel)
        assert np.array_equal(got, oracle.tdes_ecb(key, data, dec)), dec
    if name.startswith("weak") or name in ("zero", "ones"):
        # a weak key's DES is an involution, and so is EDE with three copies
        twice = _gpu(torch_dev, key, _gpu(torch_dev, key, data, kernel=kernel), kernel=kernel)
        assert np.array_equal(twice, data)
    if name == "k1_eq_k2":
        k3 = np.tile(key[16:], 3)
        assert np.array_equal(_gpu(torch_dev, key, data, kernel=kernel),
                              oracle.tdes_ecb(k3, data))


@pytest.mark.parametrize("kernel", KERNELS)
def test_side_stream(torch_dev, kernel):
    # The launch goes on the stream the caller names, not on the null stream.
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x72)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 5 * 16384 + 8 * 11)
    x = torch.from_numpy(data).cuda()
    out = torch.zeros_like(x)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    _say("side stream", kernel)
    T.encrypt(key, x, out, kernel=kernel, stream=s)
    back = torch.empty_like(x)
    T.decrypt(key, out, back, kernel=kernel, stream=s)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.tdes_ecb(key, data))
    assert torch.equal(back, x)


@pytest.mark.parametrize("kernel", KERNELS)
def test_offsets_beyond_4gib(torch_dev, kernel):
    # A buffer of 4 GiB plus three wave chunks plus 5 blocks, filled with
    # block counters (block i holds i as a little-endian 64-bit integer, so
    # an output read from or written to a wrong address cannot match).
    # Blocks around byte offsets 2^31 and 2^32, the tail and seeded random
    # positions are checked against the oracle one by one; decryption of the
    # whole output must give back every block.
    torch = torch_dev
    nblk = (4 * GIB + 3 * 16384) // 8 + 5
    key = W.key_bundle(W.rng(W.SEED_BASE + 0x73))
    _say("beyond 4GiB", kernel, nblk)
    x = torch.arange(nblk, dtype=torch.int64, device="cuda").view(torch.uint8)
    out = torch.empty_like(x)
    T.encrypt(key, x, out, kernel=kernel)
    b2, b4 = (1 << 31) // 8, (1 << 32) // 8
    idx = np.unique(np.concatenate([
        np.arange(b2 - 2048, b2 + 2048), np.arange(b4 - 4096, b4 + 4096),
        np.arange(nblk - 8192, nblk),
        W.rng(W.SEED_BASE + 0x74).choice(nblk, 1 << 15, replace=False)]))
    ti = torch.from_numpy(idx).cuda()
    got = out.view(-1, 8)[ti].cpu().numpy().reshape(-1)
    sample = x.view(-1, 8)[ti].cpu().numpy().reshape(-1)
    assert np.array_equal(sample.view(np.int64), idx)
    assert np.array_equal(got, oracle.tdes_ecb(key, sample))
    T.decrypt(key, out, out, kernel=kernel)
    same = torch.equal(out, x)
    del x, out
    assert same


@pytest.mark.parametrize("nblocks", [1, 3, 4096, 12345])
@pytest.mark.parametrize("two_key", [False, True])
def test_paper_design_matches_oracle(torch_dev, nblocks, two_key):
    # The paper's one-thread-per-bit design (three launches), both directions.
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x80 + nblocks + two_key)
    key = W.key_bundle(g, two_key=two_key)
    data = W.uniform_bytes(g, 8 * nblocks)
    _say("paper design", nblocks, "two_key", two_key)
    x = torch.from_numpy(data).cuda()
    for dec in (False, True):
        out = torch.empty_like(x)
        T.paper_design_ptr(T.key_schedule(key), T.DECRYPT if dec else T.ENCRYPT, x.data_ptr(),
                           out.data_ptr(), x.numel(), int(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), oracle.tdes_ecb(key, data, dec)), dec


def test_paper_design_64mib_equals_bitsliced(torch_dev):
    torch = torch_dev
    key, data, want = _c2_case(False)
    _say("paper design 64MiB")
    x = torch.from_numpy(data).cuda()
    out = torch.empty_like(x)
    T.paper_design_ptr(T.key_schedule(key), T.ENCRYPT, x.data_ptr(), out.data_ptr(), x.numel(),
                       int(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)


def test_valu_probes_run(torch_dev):
    # The issue-rate probes the roofline discussion rests on: every opcode
    # launches and returns a positive rate.
    from paper_2007_10752_amd import probe
    for op in probe.OPS:
        assert probe.valu_rate(op, blocks=256, iters=64, reps=1) > 0, op
