"""GPU parity of the batched form (tdes_batch_submit): many messages with
their own keys and directions in one pass, each bit-exact against the oracle
and against the plain single-message call."""
import sys

import numpy as np
import pytest

import oracle
from paper_2007_10752_amd import tdes as T
from paper_2007_10752_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run_batch(torch, keys, lengths, dirs, data, inplace=False, gap=0):
    n = len(lengths)
    offs = np.zeros(n, dtype=np.int64)
    if n > 1:
        offs[1:] = np.cumsum(np.asarray(lengths, dtype=np.int64) + gap)[:-1]
    x = torch.from_numpy(data).cuda()
    out = x if inplace else torch.full_like(x, 0xA5)
    b = T.Batch(keys, offs, offs, lengths, dirs)
    b.submit(x, out)
    torch.cuda.synchronize()
    return offs, out.cpu().numpy(), b


def test_small_mixed_batch(torch_dev):
    g = W.rng(W.SEED_BASE + 0x300)
    n = 57
    lengths = (g.integers(0, 700, size=n) * 8).astype(np.int64)
    lengths[:4] = [0, 8, 256, 264]
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    data = W.uniform_bytes(g, int(lengths.sum()))
    _say("batch small", n, int(lengths.sum()))
    offs, got, b = _run_batch(torch_dev, keys, lengths, dirs, data)
    assert b.skipped() == 0
    for i in range(n):
        seg = slice(int(offs[i]), int(offs[i] + lengths[i]))
        assert np.array_equal(got[seg], oracle.tdes_ecb(keys[i], data[seg], bool(dirs[i]))), i


def test_runs_of_empty_and_one_slice_messages(torch_dev):
    # More than 64 empty messages in a row between non-empty ones, and
    # stretches where every lane of a wave holds its own message: the cases
    # the per-lane message lookup handles by walking on past the 64 starts
    # it searches, and by the search itself.
    g = W.rng(W.SEED_BASE + 0x304)
    lengths = np.concatenate([
        [0] * 70, [256], [0] * 130, (g.integers(1, 33, size=200) * 8),
        [0] * 65, [8], [0] * 64, [4096], [0] * 3]).astype(np.int64)
    n = len(lengths)
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    data = W.uniform_bytes(g, int(lengths.sum()))
    _say("batch empty runs", n, int(lengths.sum()))
    offs, got, b = _run_batch(torch_dev, keys, lengths, dirs, data)
    assert b.skipped() == 0
    for i in range(n):
        seg = slice(int(offs[i]), int(offs[i] + lengths[i]))
        assert np.array_equal(got[seg], oracle.tdes_ecb(keys[i], data[seg], bool(dirs[i]))), i


def test_in_place_and_gaps(torch_dev):
    g = W.rng(W.SEED_BASE + 0x301)
    n = 20
    lengths = (g.integers(1, 300, size=n) * 8).astype(np.int64)
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    gap = 24
    total = int(lengths.sum()) + gap * n
    data = W.uniform_bytes(g, total)
    offs, got, _ = _run_batch(torch_dev, keys, lengths, dirs, data, inplace=True, gap=gap)
    for i in range(n):
        seg = slice(int(offs[i]), int(offs[i] + lengths[i]))
        assert np.array_equal(got[seg], oracle.tdes_ecb(keys[i], data[seg], bool(dirs[i]))), i
        gseg = slice(int(offs[i] + lengths[i]), int(offs[i] + lengths[i] + gap))
        assert np.array_equal(got[gseg], data[gseg]), "gap bytes were written"


def test_single_message_waves(torch_dev):
    # Waves whose 64 slices lie in one message take the coalesced path
    # (buffer resource sized to the bytes left in the message); the others
    # read their slices 16 bytes at a time, clamped to the slice.  Messages
    # of whole waves, of a wave plus 8 bytes, of odd block counts and of one
    # block, at offsets that are multiples of 8 but not of 16, both in one
    # batch and each alone (then every wave of it is single-message).
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x305)
    lengths = np.array([16384, 16392, 3 * 16384 + 8, (1 << 20) + 8, 8, 264, 40, 16, 24,
                        2 * 16384 - 8], dtype=np.int64)
    n = len(lengths)
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    gap = 8
    offs = np.zeros(n, dtype=np.int64)
    offs[1:] = np.cumsum(lengths + gap)[:-1]
    offs += 8  # 8-byte aligned, not 16-byte aligned
    total = int(offs[-1] + lengths[-1] + 8)
    data = W.uniform_bytes(g, total)
    x = torch.from_numpy(data).cuda()
    want = data.copy()
    for i in range(n):
        seg = slice(int(offs[i]), int(offs[i] + lengths[i]))
        want[seg] = oracle.tdes_ecb(keys[i], data[seg], bool(dirs[i]))
    _say("batch single-message waves", n, total)
    out = x.clone()
    T.Batch(keys, offs, offs, lengths, dirs).submit(x, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    for i in range(n):
        out = x.clone()
        T.Batch(keys[i:i + 1], offs[i:i + 1], offs[i:i + 1], lengths[i:i + 1],
                dirs[i:i + 1]).submit(x, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        seg = slice(int(offs[i]), int(offs[i] + lengths[i]))
        assert np.array_equal(got[seg], want[seg]), i
        rest = np.ones(total, dtype=bool)
        rest[seg] = False
        assert np.array_equal(got[rest], data[rest]), ("bytes outside the message changed", i)


def test_invalid_messages_are_skipped(torch_dev):
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x302)
    keys = W.key_bundles(g, 3)
    data = W.uniform_bytes(g, 4096)
    x = torch.from_numpy(data).cuda()
    out = torch.zeros_like(x)
    # message 1 has a length that is not a multiple of 8, message 2 a bad schedule
    b = T.Batch(keys, [0, 1024, 2048], [0, 1024, 2048], [1024, 1020, 1024], [0, 0, 1],
                sched_idx=[0, 1, 2])
    b.msgs[2, 3] = (7 | (1 << 32))  # schedule index 7 of 3
    b.submit(x, out)
    torch.cuda.synchronize()
    assert b.skipped() == 2
    got = out.cpu().numpy()
    assert np.array_equal(got[:1024], oracle.tdes_ecb(keys[0], data[:1024]))
    assert not got[1024:].any()


def test_16k_lognormal_batch(torch_dev):
    torch = torch_dev
    lay = W.batched_layout(W.SEED_BASE + 3)
    g = W.rng(W.SEED_BASE + 3 + W.KEY_SEED_OFFSET)
    data = W.uniform_bytes(g, lay["total"])
    _say("batch 16384 messages,", lay["total"], "bytes")
    x = torch.from_numpy(data).cuda()
    out = torch.empty_like(x)
    b = T.Batch(lay["keys"], lay["offsets"], lay["offsets"], lay["lengths"], lay["dirs"])
    b.submit(x, out)
    torch.cuda.synchronize()
    assert b.skipped() == 0
    got = out.cpu().numpy()
    # every message equals the plain single-message path ...
    sch = T.key_schedules(lay["keys"])
    plain = torch.empty_like(x)
    for i in range(len(lay["lengths"])):
        o, n = int(lay["offsets"][i]), int(lay["lengths"][i])
        T.ecb(sch[i], x[o:o + n], plain[o:o + n], decrypt=bool(lay["dirs"][i]))
    torch.cuda.synchronize()
    assert torch.equal(out, plain)
    # ... and a seeded sample of messages equals the oracle
    pick = W.rng(W.SEED_BASE + 0x303).choice(len(lay["lengths"]), 512, replace=False)
    for i in pick:
        o, n = int(lay["offsets"][i]), int(lay["lengths"][i])
        want = oracle.tdes_ecb(lay["keys"][i], data[o:o + n], bool(lay["dirs"][i]))
        assert np.array_equal(got[o:o + n], want), i


@pytest.mark.parametrize("n", [1, 1023, 1024, 1025, 8191, 8192, 8193, 20000])
def test_scan_chunk_boundaries(torch_dev, n):
    # The descriptor scan works in tiles of 1024 messages (one workgroup
    # each, then tile offsets): batches just below, at and just above tile
    # edges, and ones spanning many tiles, with short messages (one to three
    # slices) and some empty ones.  The first-slice table is compared whole
    # with the prefix sums of the slice counts.
    g = W.rng(W.SEED_BASE + 0x305 + n)
    lengths = (g.integers(0, 97, size=n) * 8).astype(np.int64)
    lengths[g.random(n) < 0.05] = 0
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    data = W.uniform_bytes(g, max(int(lengths.sum()), 8))
    _say("batch scan edges", n, int(lengths.sum()))
    offs, got, b = _run_batch(torch_dev, keys, lengths, dirs, data)
    assert b.skipped() == 0
    slices = (lengths + 255) // 256
    first = np.concatenate([[0], np.cumsum(slices)]).astype(np.int64)
    table = b.ws.cpu().numpy()
    assert table[0] == first[-1] and table[1] == 0
    assert np.array_equal(table[2:2 + n + 1], first)
    if n < 64:
        check = range(n)
    else:
        sample = W.rng(W.SEED_BASE + 0x306).choice(n, 64, replace=False).tolist()
        check = sorted(set(sample) | {0, n - 1, min(8191, n - 1), min(8192, n - 1)})
    for i in check:
        seg = slice(int(offs[i]), int(offs[i] + lengths[i]))
        assert np.array_equal(got[seg], oracle.tdes_ecb(keys[i], data[seg], bool(dirs[i]))), i


def test_scan_beyond_fused_tiles(torch_dev):
    # More than 8192 tiles of 1024 descriptors: the tile offsets are then
    # scanned by one workgroup and added by a third launch.  8,388,613
    # one-block messages sharing two schedules; the whole first-slice table
    # is compared with the prefix sums, and a sample of messages with the
    # oracle.
    torch = torch_dev
    n = 8192 * 1024 + 5
    g = W.rng(W.SEED_BASE + 0x30E)
    keys = W.key_bundles(g, 2)
    sch = T.key_schedules(keys)
    d_sched = torch.empty(2 * T.DEVICE_SCHEDULE_BYTES, dtype=torch.uint8, device="cuda")
    T.schedule_upload(sch, d_sched.data_ptr(), T._stream_handle(None))
    offs = np.arange(n, dtype=np.int64) * 8
    idx = np.arange(n) % 2
    msgs = torch.from_numpy(T.msg_table(offs, offs, np.full(n, 8), idx, idx)).cuda()
    data = W.uniform_bytes(g, 8 * n)
    x = torch.from_numpy(data).cuda()
    out = torch.zeros_like(x)
    ws_bytes = T.batch_workspace_bytes(n)
    ws = torch.empty((ws_bytes + 7) // 8, dtype=torch.int64, device="cuda")
    _say("batch scan beyond fused tiles", n)
    T.batch_submit_ptr(msgs.data_ptr(), n, d_sched.data_ptr(), 2, x.data_ptr(), x.numel(),
                       out.data_ptr(), out.numel(), ws.data_ptr(), ws_bytes)
    torch.cuda.synchronize()
    table = ws.cpu().numpy()
    assert table[0] == n and table[1] == 0
    assert np.array_equal(table[2:2 + n + 1], np.arange(n + 1))
    got = out.cpu().numpy()
    for i in W.rng(W.SEED_BASE + 0x30F).choice(n, 256, replace=False).tolist() + [0, n - 1]:
        seg = slice(8 * i, 8 * i + 8)
        assert np.array_equal(got[seg], oracle.tdes_ecb(keys[i % 2], data[seg], bool(i % 2))), i


def test_offsets_beyond_4gib(torch_dev):
    # Input offsets that straddle byte 2^32 of the input base, outputs at
    # different (low) offsets of another base.
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x307)
    n = 300
    lengths = (g.integers(0, 200, size=n) * 8).astype(np.int64)
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    total = int(lengths.sum())
    rel = np.zeros(n, dtype=np.int64)
    rel[1:] = np.cumsum(lengths)[:-1]
    start = ((1 << 32) - total // 2) & ~7
    data = W.uniform_bytes(g, total)
    _say("batch beyond 4GiB", n, total, start)
    x = torch.empty(start + total, dtype=torch.uint8, device="cuda")
    x[start:].copy_(torch.from_numpy(data))
    out = torch.full((total,), 0xA5, dtype=torch.uint8, device="cuda")
    b = T.Batch(keys, start + rel, rel, lengths, dirs)
    b.submit(x, out)
    torch.cuda.synchronize()
    assert b.skipped() == 0
    got = out.cpu().numpy()
    del x, out
    for i in range(n):
        seg = slice(int(rel[i]), int(rel[i] + lengths[i]))
        assert np.array_equal(got[seg], oracle.tdes_ecb(keys[i], data[seg], bool(dirs[i]))), i


def test_device_key_expansion_matches_host(torch_dev):
    """tdes_schedule_expand (key generation on the GPU) writes exactly the
    bytes tdes_schedule_upload writes from the host key schedule."""
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x304)
    n = 777
    keys = W.key_bundles(g, n)
    keys[5] = np.repeat(keys[5][:8][None], 3, axis=0).reshape(-1)  # K1 = K2 = K3
    a = torch.zeros(n * T.DEVICE_SCHEDULE_BYTES, dtype=torch.uint8, device="cuda")
    b = torch.ones_like(a)
    T.schedule_upload(T.key_schedules(keys), a.data_ptr(), int(torch.cuda.current_stream().cuda_stream))
    dk = torch.from_numpy(np.ascontiguousarray(keys)).cuda()
    T.schedule_expand(dk.data_ptr(), n, b.data_ptr(), int(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_batch_replays_in_a_captured_graph(torch_dev):
    # The batched call only enqueues kernels on the caller's stream (no
    # memset, no allocation, no synchronisation), so it can be captured in a
    # HIP graph.  Each replay, with eager work and a new input in between,
    # must equal the eager result on the same input.
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x308)
    n = 300
    lengths = (g.integers(0, 120, size=n) * 8).astype(np.int64)
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    total = int(lengths.sum())
    offs = np.zeros(n, dtype=np.int64)
    offs[1:] = np.cumsum(lengths)[:-1]
    x = torch.from_numpy(W.uniform_bytes(g, total)).cuda()
    out = torch.empty_like(x)
    b = T.Batch(keys, offs, offs, lengths, dirs)
    b.submit(x, out)  # eager first: one-time set-up happens outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.submit(x, out, stream=torch.cuda.current_stream())
    _say("batch graph replays")
    for r in range(3):
        x.copy_(torch.from_numpy(W.uniform_bytes(W.rng(W.SEED_BASE + 0x309 + r), total)))
        out.fill_(r)
        want = torch.full_like(x, 0xA5)
        b.submit(x, want)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), r
        assert b.skipped() == 0
    got = out.cpu().numpy()
    data = x.cpu().numpy()
    for i in range(0, n, 37):
        seg = slice(int(offs[i]), int(offs[i] + lengths[i]))
        assert np.array_equal(got[seg], oracle.tdes_ecb(keys[i], data[seg], bool(dirs[i]))), i


@pytest.fixture(autouse=True)
def _tune_cache(tmp_path, monkeypatch):
    # the tuner's cache file goes to a scratch path, never the user's cache
    monkeypatch.setenv("TDES_TUNE_CACHE", str(tmp_path / "tune.json"))


def test_every_configuration_gives_the_same_bytes(torch_dev):
    # Every compiled variant (messages per mask table x waves per SIMD) at
    # every grid multiplier: the same output, equal to the oracle's.  The
    # batch mixes many tiny messages (waves spanning more messages than one
    # mask table holds) with longer ones.
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x30D)
    n = 700
    lengths = np.where(g.random(n) < 0.7, g.integers(1, 9, size=n) * 8,
                       g.integers(1, 600, size=n) * 8).astype(np.int64)
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    data = W.uniform_bytes(g, int(lengths.sum()))
    offs, want, b = _run_batch(torch, keys, lengths, dirs, data)
    for i in range(0, n, 7):
        seg = slice(int(offs[i]), int(offs[i] + lengths[i]))
        assert np.array_equal(want[seg], oracle.tdes_ecb(keys[i], data[seg], bool(dirs[i]))), i
    x = torch.from_numpy(data).cuda()
    keep = T.batch_get_config()
    try:
        # the compiled variants (tdes_batch_config in include/tdes.h)
        for kmax, waves in ((8, 4), (4, 4), (8, 3), (4, 3), (16, 3), (8, 5), (4, 5)):
            for mult in (1, 2, 3, 4):
                _say("batch config", kmax, waves, mult)
                T.batch_set_config(kmax, waves, mult)
                out = torch.full_like(x, 0xA5)
                b.submit(x, out)
                torch.cuda.synchronize()
                assert np.array_equal(out.cpu().numpy(), want), (kmax, waves, mult)
    finally:
        T.batch_set_config(keep["kmax"], keep["waves"], keep["grid_mult"])


def test_autotune_writes_the_cache(torch_dev, tmp_path):
    # The winner is written under this device's architecture name and CU
    # count; loading that entry gives the configuration now in use.
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x30E)
    n = 200
    lengths = (g.integers(1, 300, size=n) * 8).astype(np.int64)
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    data = W.uniform_bytes(g, int(lengths.sum()))
    offs, want, b = _run_batch(torch, keys, lengths, dirs, data)
    x = torch.from_numpy(data).cuda()
    out = torch.empty_like(x)
    m = b.autotune(x, out, reps=1)
    assert m["saved"] == 1
    prop = torch.cuda.get_device_properties(0)
    got = T.batch_config_load(str(tmp_path / "tune.json"), prop.gcnArchName,
                              prop.multi_processor_count)
    assert got is not None, open(str(tmp_path / "tune.json")).read()
    assert (got["kmax"], got["waves"], got["grid_mult"]) == (m["kmax"], m["waves"], m["grid_mult"])
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)


def test_batch_autotune_keeps_results(torch_dev):
    # The autotuner runs the batch at several grids; every run, and every
    # later submit at the chosen grid, gives the same bytes.
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x30A)
    n = 500
    lengths = (g.integers(0, 200, size=n) * 8).astype(np.int64)
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    total = int(lengths.sum())
    data = W.uniform_bytes(g, total)
    offs, want, b = _run_batch(torch, keys, lengths, dirs, data)
    x = torch.from_numpy(data).cuda()
    out = torch.full_like(x, 0xA5)
    _say("batch autotune")
    m = b.autotune(x, out, reps=2)
    assert m["grid_mult"] in (1, 2, 3, 4) and m["kmax"] in (4, 8, 16) and m["waves"] in (3, 4, 5)
    cur = T.batch_get_config()
    assert (cur["kmax"], cur["waves"], cur["grid_mult"]) == (m["kmax"], m["waves"], m["grid_mult"])
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    out2 = torch.full_like(x, 0x5A)
    b.submit(x, out2)
    torch.cuda.synchronize()
    assert np.array_equal(out2.cpu().numpy(), want)
    for i in range(0, n, 53):
        seg = slice(int(offs[i]), int(offs[i] + lengths[i]))
        assert np.array_equal(want[seg], oracle.tdes_ecb(keys[i], data[seg], bool(dirs[i]))), i


def test_batch_autotune_streams_keeps_results(torch_dev):
    # The stream-of-batches autotuner runs the batch on two streams at once,
    # each lane into its own output with its own workspace: both outputs hold
    # the batch's bytes, and the kept configuration is the current one.
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x30D)
    n = 300
    lengths = (g.integers(0, 300, size=n) * 8).astype(np.int64)
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    data = W.uniform_bytes(g, int(lengths.sum()))
    offs, want, b = _run_batch(torch, keys, lengths, dirs, data)
    x = torch.from_numpy(data).cuda()
    outs = [torch.full_like(x, 0xA5), torch.full_like(x, 0x5A)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    _say("batch autotune, two streams")
    m = b.autotune_streams(x, outs, streams, reps=2)
    assert m["grid_mult"] in (1, 2, 3, 4) and m["kmax"] in (4, 8, 16) and m["waves"] in (3, 4, 5)
    cur = T.batch_get_config()
    assert (cur["kmax"], cur["waves"], cur["grid_mult"]) == (m["kmax"], m["waves"], m["grid_mult"])
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(o.cpu().numpy(), want)
    for i in range(0, n, 37):
        seg = slice(int(offs[i]), int(offs[i] + lengths[i]))
        assert np.array_equal(want[seg], oracle.tdes_ecb(keys[i], data[seg], bool(dirs[i]))), i


def test_out_of_range_messages_are_skipped(torch_dev):
    # Message ranges are checked against the input and output buffer sizes:
    # a message reaching past either end (including offsets that would wrap
    # a 64-bit sum) is skipped and counted, and nothing past the declared
    # output size is written.
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x30B)
    keys = W.key_bundles(g, 6)
    data = W.uniform_bytes(g, 8192)
    x = torch.from_numpy(data).cuda()
    big = torch.full((8192 + 4096,), 0x3C, dtype=torch.uint8, device="cuda")
    out = big[:8192]
    in_off = [0, 4096, 8192 - 512, 1024, (1 << 64) - 8, 2048]
    out_off = [0, 4096, 2048, 8192 - 256, 512, (1 << 64) - 1024]
    lengths = [1024, 1024, 1024, 512, 64, 1024]
    # 2: input past the end; 3: output past the end; 4: input offset wraps;
    # 5: output offset wraps
    b = T.Batch(keys, np.array(in_off, dtype=np.uint64).astype(np.int64),
                np.array(out_off, dtype=np.uint64).astype(np.int64), lengths, [0, 1, 0, 0, 0, 0])
    b.submit(x, out)
    torch.cuda.synchronize()
    assert b.skipped() == 4
    got = big.cpu().numpy()
    assert np.array_equal(got[:1024], oracle.tdes_ecb(keys[0], data[:1024]))
    assert np.array_equal(got[4096:5120], oracle.tdes_ecb(keys[1], data[4096:5120], True))
    untouched = np.ones(got.size, bool)
    untouched[:1024] = False
    untouched[4096:5120] = False
    assert (got[untouched] == 0x3C).all()


def test_autotune_refuses_aliasing_buffers(torch_dev):
    # Every trial of the autotuner rewrites the output from the input, so an
    # in-place batch would be encrypted once per trial: it is refused.
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x30C)
    n = 40
    lengths = (g.integers(1, 100, size=n) * 8).astype(np.int64)
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    data = W.uniform_bytes(g, int(lengths.sum()))
    offs, want, b = _run_batch(torch, keys, lengths, dirs, data)
    x = torch.from_numpy(data).cuda()
    with pytest.raises(T.TdesError) as e:
        b.autotune(x, x, reps=1)
    assert e.value.status == -4
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), data)  # nothing ran
