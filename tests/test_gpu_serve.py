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
    torch, pool, arena, pad = env
    got = {}

    def keep(comp):
        for c in comp:
            t = int(c["tag"])
            if t in capture and c["status"] == 0:
                off = int(c["d_out"]) - arena.data_ptr()
                got[t] = arena[off: off + int(c["nbytes"])].cpu().numpy()

    lat, status, wall, st = S.run_open_loop(srv, reqs, arrival, on_complete=keep)
    return got, lat, status, st


def _pool_bytes(env, r):
    torch, pool, arena, pad = env
    off = int(r["d_in"]) - pool.data_ptr()
    return pool[off: off + int(r["nbytes"])].cpu().numpy()


@pytest.mark.parametrize("mode", [S.BATCHED, S.PLAIN])
def test_mixed_equals_alone_and_oracle(env, mode):
    torch, pool, arena, pad = env
    trace = W.serving_trace(W.SEED_BASE + 5, rate=20000, duration_s=0.15, bands=SMALL_BANDS)
    reqs = S.make_requests(trace, pool.data_ptr(), pool.numel(), W.SEED_BASE + 6)
    n = len(reqs)
    capture = set(W.rng(W.SEED_BASE + 7).choice(n, 48, replace=False).tolist())
    capture |= {int(np.argmax(trace["size"]))}
    _say("serve mix mode", mode, n, "requests")
    srv = _server(env, mode=mode, slots=4, max_batch_msgs=1024)
    got, lat, status, st = _run(env, srv, reqs, trace["arrival"], capture)
    srv.close()
    assert (status == 0).all()
    assert st["completed"] == n and st["released"] == n and st["in_flight_bytes"] == 0
    if mode == S.BATCHED:
        assert st["batches"] < n                 # requests really were batched
    alone = _server(env, mode=S.BATCHED, slots=1, max_batch_msgs=1)
    for t in sorted(capture):
        one, _, st1, _ = _run(env, alone, reqs[t:t + 1], np.zeros(1), {0})
        assert (st1 == 0).all()
        assert np.array_equal(one[0], got[t]), t
        want = oracle.tdes_ecb(trace["keys"][t], _pool_bytes(env, reqs[t]), bool(trace["dirs"][t]))
        assert np.array_equal(got[t], want), t
    alone.close()


def test_budget_holds_under_load(env):
    budget = 6 << 20
    trace = W.serving_trace(W.SEED_BASE + 8, rate=50000, duration_s=0.05, bands=SMALL_BANDS)
    torch, pool, arena, pad = env
    reqs = S.make_requests(trace, pool.data_ptr(), pool.numel(), W.SEED_BASE + 9)
    srv = _server(env, budget_bytes=budget, slots=4, max_batch_msgs=256)
    _, lat, status, st = _run(env, srv, reqs, trace["arrival"], set())
    srv.close()
    assert (status == 0).all()
    assert st["peak_in_flight_bytes"] <= budget
    assert st["completed"] == len(reqs)
