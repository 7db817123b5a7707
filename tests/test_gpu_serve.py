"""GPU tests of the request server: results served in a mix of concurrent
requests equal the same requests served alone and the oracle, bit for bit,
and the in-flight budget holds under load."""
import sys

import numpy as np
import pytest

import oracle
from paper_2007_10752_amd import serve as S
from paper_2007_10752_amd import workloads as W

pytestmark = pytest.mark.gpu

SMALL_BANDS = ((0.70, 64, 1024), (0.25, 4096, 65536), (0.05, 1 << 18, 1 << 20))


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gen = torch.Generator(device="cuda").manual_seed(W.SEED_BASE + 4)
    pool = torch.randint(0, 256, (64 << 20,), dtype=torch.uint8, device="cuda", generator=gen)
    arena = torch.empty((256 << 20) + 256, dtype=torch.uint8, device="cuda")
    pad = (-arena.data_ptr()) % 256
    return torch, pool, arena, pad


def _server(env, **kw):
    torch, pool, arena, pad = env
    return S.Server(arena.data_ptr() + pad, 256 << 20, **kw)


def _run(env, srv, reqs, arrival, capture):
    """Serve the trace; keep a device copy of the results whose tags are in
    capture (None: all) and the batch number each request ran in."""
    torch, pool, arena, pad = env
    got, batch_of = {}, {}

    def keep(comp):
        copied = False
        for c in comp:
            t = int(c["tag"])
            batch_of[t] = int(c["batch"])
            if (capture is None or t in capture) and c["status"] == 0:
                off = int(c["d_out"]) - arena.data_ptr()
                got[t] = arena[off: off + int(c["nbytes"])].clone()
                copied = True
        if copied:
            # the driver releases these results next: the copies (on torch's
            # stream) must be done before the server reuses their arena space
            torch.cuda.current_stream().synchronize()

    lat, status, wall, st = S.run_open_loop(srv, reqs, arrival, on_complete=keep)
    return got, lat, status, st, batch_of


def _pool_bytes(env, r):
    torch, pool, arena, pad = env
    off = int(r["d_in"]) - pool.data_ptr()
    return pool[off: off + int(r["nbytes"])].cpu().numpy()


@pytest.mark.parametrize("mode", [S.BATCHED, S.PLAIN])
def test_mixed_equals_alone_and_oracle(env, mode):
    torch, pool, arena, pad = env
    # 100k requests/s: enough concurrency that many batches hold more than the
    # three small requests the server runs as separate plain launches
    trace = W.serving_trace(W.SEED_BASE + 5, rate=100000, duration_s=0.03, bands=SMALL_BANDS)
    reqs = S.make_requests(trace, pool.data_ptr(), pool.numel(), W.SEED_BASE + 6)
    n = len(reqs)
    # the first 64 arrive together: they queue before the first launch and
    # share one batch whatever the host's speed, so batch-kernel output is
    # always among the checked results
    arrival = trace["arrival"].copy()
    arrival[:64] = 0.0
    _say("serve mix mode", mode, n, "requests")
    srv = _server(env, mode=mode, slots=4, max_batch_msgs=1024)
    got, lat, status, st, batch_of = _run(env, srv, reqs, arrival, None)
    srv.close()
    assert (status == 0).all()
    assert st["completed"] == n and st["released"] == n and st["in_flight_bytes"] == 0
    # checked: requests that shared a batch of more than three (in batched
    # mode the batch kernel ran them, the property continuous batching must
    # keep; smaller batches of small requests run as plain launches),
    # requests that ran alone, and the largest request
    size = {}
    for b in batch_of.values():
        size[b] = size.get(b, 0) + 1
    shared = [t for t in range(n) if size[batch_of[t]] > 3]
    few = [t for t in range(n) if 1 < size[batch_of[t]] <= 3]
    single = [t for t in range(n) if size[batch_of[t]] == 1]
    pick = W.rng(W.SEED_BASE + 7)
    capture = set(pick.choice(shared, min(40, len(shared)), replace=False).tolist()) if shared else set()
    capture |= set(pick.choice(few, min(16, len(few)), replace=False).tolist()) if few else set()
    capture |= set(pick.choice(single, min(8, len(single)), replace=False).tolist()) if single else set()
    capture |= {int(np.argmax(trace["size"]))}
    if mode == S.BATCHED:
        assert st["batches"] < n                 # requests really were batched
        assert len(shared) >= 40, len(shared)    # and the check covers batch-kernel output
    _say("serve mix shared/few/single", len(shared), len(few), len(single))
    alone = _server(env, mode=S.BATCHED, slots=1, max_batch_msgs=1)
    for t in sorted(capture):
        one, _, st1, _, _ = _run(env, alone, reqs[t:t + 1], np.zeros(1), {0})
        assert (st1 == 0).all()
        mine = got[t].cpu().numpy()
        assert np.array_equal(one[0].cpu().numpy(), mine), t
        want = oracle.tdes_ecb(trace["keys"][t], _pool_bytes(env, reqs[t]), bool(trace["dirs"][t]))
        assert np.array_equal(mine, want), t
    alone.close()


def test_budget_holds_under_load(env):
    budget = 6 << 20
    trace = W.serving_trace(W.SEED_BASE + 8, rate=50000, duration_s=0.05, bands=SMALL_BANDS)
    torch, pool, arena, pad = env
    reqs = S.make_requests(trace, pool.data_ptr(), pool.numel(), W.SEED_BASE + 9)
    srv = _server(env, budget_bytes=budget, slots=4, max_batch_msgs=256)
    _, lat, status, st, _ = _run(env, srv, reqs, trace["arrival"], set())
    srv.close()
    assert (status == 0).all()
    assert st["peak_in_flight_bytes"] <= budget
    assert st["completed"] == len(reqs)


# One burst per case, one slot: the whole burst is one batch.  Batches of 4 to
# 64 requests and at most 4 MiB run as one table-kernel launch over the
# requests, larger ones on the batched bitsliced path; every result is
# compared with the oracle.
TABLE_BANDS = ((0.70, 64, 1024), (0.30, 4096, 65536))


@pytest.mark.parametrize("count,bands", [(4, TABLE_BANDS), (17, TABLE_BANDS), (64, TABLE_BANDS),
                                         (65, TABLE_BANDS), (4, ((1.0, 1 << 20, 1 << 20),)),
                                         (8, ((1.0, 1 << 20, 1 << 20),))])
def test_burst_batches_equal_oracle(env, count, bands):
    trace = W.serving_trace(W.SEED_BASE + 10 + count, rate=100000, duration_s=0.01, bands=bands)
    assert len(trace["size"]) >= count
    trace = {k: v[:count] for k, v in trace.items()}
    torch, pool, arena, pad = env
    reqs = S.make_requests(trace, pool.data_ptr(), pool.numel(), W.SEED_BASE + 11)
    _say("serve burst", count, int(trace["size"].sum()), "bytes")
    srv = _server(env, slots=1, max_batch_msgs=1024)
    got, lat, status, st, batch_of = _run(env, srv, reqs, np.zeros(count), None)
    srv.close()
    assert (status == 0).all()
    assert st["batches"] == 1, st["batches"]
    for t in range(count):
        want = oracle.tdes_ecb(trace["keys"][t], _pool_bytes(env, reqs[t]), bool(trace["dirs"][t]))
        assert np.array_equal(got[t].cpu().numpy(), want), t


# Bursts of small requests with a few large ones (above 4 MiB in all, some
# requests above the table kernel's one-pass size): the batched path.
@pytest.mark.parametrize("big", [[(2, 5 << 19), (5, 5 << 19), (7, 5 << 19)],
                                 [(3, 6 << 20)],
                                 [(0, 2 << 20), (1, 2 << 20), (2, 2 << 20), (3, 2 << 20), (4, 2 << 20)]])
def test_burst_with_large_requests(env, big):
    count = 12
    trace = W.serving_trace(W.SEED_BASE + 40 + len(big), rate=100000, duration_s=0.01,
                            bands=TABLE_BANDS)
    trace = {k: v[:count].copy() for k, v in trace.items()}
    for i, nbytes in big:
        trace["size"][i] = nbytes
    torch, pool, arena, pad = env
    reqs = S.make_requests(trace, pool.data_ptr(), pool.numel(), W.SEED_BASE + 12)
    _say("serve burst with large", [b for _, b in big], int(trace["size"].sum()), "bytes")
    srv = _server(env, slots=1, max_batch_msgs=1024)
    got, lat, status, st, batch_of = _run(env, srv, reqs, np.zeros(count), None)
    srv.close()
    assert (status == 0).all()
    assert st["batches"] == 1, st["batches"]
    for t in range(count):
        want = oracle.tdes_ecb(trace["keys"][t], _pool_bytes(env, reqs[t]), bool(trace["dirs"][t]))
        assert np.array_equal(got[t].cpu().numpy(), want), t
