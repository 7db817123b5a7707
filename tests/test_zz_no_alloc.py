"""The batched call without a workspace (tdes_batch_submit_noalloc): its
scan table lives in a fixed device array of the library, so the call
allocates nothing.  On the GPU its output must equal tdes_batch_submit's on
the same batch, bit for bit, on two calls in a row (the second smaller, so
it runs over what the first left in the array), and the oracle on a sample
of messages."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2007_10752_amd import tdes as T
from paper_2007_10752_amd import workloads as W


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_noalloc_rejects_more_messages_than_its_array_holds():
    # checked on the host before any device work (the pointers are never used)
    st = T.lib().tdes_batch_submit_noalloc(
        ctypes.c_void_p(8), T.BATCH_NOALLOC_MAX_MSGS + 1, ctypes.c_void_p(16), 1,
        ctypes.c_void_p(8), 8, ctypes.c_void_p(8), 8, None, None)
    assert st == -1  # TDES_ERR_ARG
    assert b"at most" in T.lib().tdes_last_error()


def test_noalloc_misaligned_skipped_counter_is_refused():
    st = T.lib().tdes_batch_submit_noalloc(
        ctypes.c_void_p(8), 1, ctypes.c_void_p(16), 1, ctypes.c_void_p(8), 8,
        ctypes.c_void_p(8), 8, ctypes.c_void_p(12), None)
    assert st == -3  # TDES_ERR_ALIGN


def _batch(seed, n, max_blocks):
    g = W.rng(seed)
    lengths = (g.integers(0, max_blocks, size=n) * 8).astype(np.int64)
    lengths[:3] = [0, 8, 256]
    keys = W.key_bundles(g, n)
    dirs = g.integers(0, 2, size=n)
    offs = np.zeros(n, dtype=np.int64)
    offs[1:] = np.cumsum(lengths)[:-1]
    data = W.uniform_bytes(g, int(lengths.sum()))
    return keys, offs, lengths, dirs, data


@pytest.mark.gpu
def test_noalloc_matches_workspace_call_twice():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for call, (seed, n, max_blocks) in enumerate(((W.SEED_BASE + 0x3A0, 900, 5000),
                                                  (W.SEED_BASE + 0x3A1, 70, 700))):
        keys, offs, lengths, dirs, data = _batch(seed, n, max_blocks)
        _say("noalloc call", call, "messages", n, "bytes", int(lengths.sum()))
        x = torch.from_numpy(data).cuda()
        b = T.Batch(keys, offs, offs, lengths, dirs)
        # one invalid message (length not a multiple of 8): skipped by both
        bad = n // 2
        b.msgs[bad, 2] = int(lengths[bad]) + 4 if lengths[bad] > 0 else 4
        ref = torch.full_like(x, 0x5A)
        b.submit(x, ref)
        new = torch.full_like(x, 0x5A)
        skipped = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        T.batch_submit_noalloc_ptr(b.msgs.data_ptr(), b.n_msgs, b.sched.data_ptr(), b.n_sched,
                                   x.data_ptr(), x.numel(), new.data_ptr(), new.numel(),
                                   skipped.data_ptr(), b.stream)
        torch.cuda.synchronize()
        assert b.skipped() == 1
        assert int(skipped.item()) == 1
        assert torch.equal(new, ref)
        got = new.cpu().numpy()
        pick = W.rng(seed + 1).choice(n, min(n, 64), replace=False)
        for i in pick:
            o, m = int(offs[i]), int(lengths[i])
            if i == bad:
                assert (got[o:o + m] == 0x5A).all(), "skipped message was written"
                continue
            want = oracle.tdes_ecb(keys[i], data[o:o + m], bool(dirs[i]))
            assert np.array_equal(got[o:o + m], want), (call, i)
