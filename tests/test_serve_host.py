"""The request server's scheduling, admission and memory accounting, run in
its host test mode (no device work: a batch completes after a fixed number
of progress calls), so these need no GPU."""
import numpy as np
import pytest

from paper_2007_10752_amd import serve as S
from paper_2007_10752_amd import tdes as T

FAKE_ARENA = 1 << 40  # never dereferenced in HOST_TEST mode


def _reqs(sizes, dirs=None, base=1 << 30):
    n = len(sizes)
    r = np.zeros(n, dtype=S.REQUEST)
    r["d_in"] = base + np.arange(n, dtype=np.uint64) * np.uint64(1 << 24)
    r["nbytes"] = sizes
    r["dir"] = 0 if dirs is None else dirs
    r["tag"] = np.arange(n)
    return r


def _server(**kw):
    args = dict(arena_ptr=FAKE_ARENA, arena_bytes=1 << 20, mode=S.HOST_TEST, slots=2,
                max_batch_msgs=8, test_polls=2)
    args.update(kw)
    return S.Server(**args)


def test_batches_complete_after_polls_and_in_order():
    s = _server()
    s.submit(_reqs([64] * 5))
    assert len(s.progress()) == 0            # admitted and launched
    st = s.stats()
    assert st["admitted"] == 5 and st["batches"] == 1 and st["busy_slots"] == 1
    c = s.progress()                          # second poll: done
    assert list(c["tag"]) == [0, 1, 2, 3, 4]
    assert (c["status"] == 0).all() and (c["batch"] == 0).all()
    assert len(set(c["d_out"].tolist())) == 5
    for d in c["d_out"]:
        s.release(d)
    st = s.stats()
    assert st["in_flight_bytes"] == 0 and st["arena_used_bytes"] == 0 and st["released"] == 5


def test_continuous_batching_over_slots():
    s = _server(slots=3, max_batch_msgs=4, test_polls=3)
    s.submit(_reqs([256] * 4))
    s.progress()                              # batch 0 on slot 0
    s.submit(_reqs([256] * 4))                # arrives while batch 0 runs
    s.progress()                              # batch 1 on slot 1
    assert s.stats()["busy_slots"] == 2
    got = []
    for _ in range(6):
        got.append(s.progress())
    c = np.concatenate(got)
    assert sorted(set(c["batch"].tolist())) == [0, 1]
    assert s.stats()["peak_busy_slots"] == 2


def test_admission_respects_budget_fifo():
    # budget 4 KiB in flight (input + output); each request 1 KiB + 1 KiB
    s = _server(budget_bytes=4096, slots=4, max_batch_msgs=16, test_polls=1)
    s.submit(_reqs([1024] * 6))
    peak = 0
    order = []
    for _ in range(20):
        c = s.progress()
        st = s.stats()
        peak = max(peak, st["in_flight_bytes"])
        assert st["in_flight_bytes"] <= 4096
        order += c["tag"].tolist()
        for d in c["d_out"]:
            s.release(d)
        if len(order) == 6:
            break
    assert order == [0, 1, 2, 3, 4, 5]        # arrival order kept
    assert s.stats()["peak_in_flight_bytes"] <= 4096
    assert s.stats()["batches"] >= 3          # at most 2 requests fit at once


def test_output_stays_reserved_until_release():
    s = _server(arena_bytes=1024, budget_bytes=1 << 20, slots=2, test_polls=1)
    s.submit(_reqs([1024, 512]))
    c = s.progress()
    c = np.concatenate([c, s.progress()])
    assert c["tag"].tolist() == [0]           # the second waits for arena space
    assert s.stats()["queued"] == 1
    s.release(c["d_out"][0])
    c2 = np.concatenate([s.progress(), s.progress()])
    assert c2["tag"].tolist() == [1]


def test_rejections_and_empty_requests():
    s = _server(arena_bytes=4096, budget_bytes=8192)
    r = _reqs([12, 8192, 0, 64, 64], dirs=[0, 0, 0, 5, 1])
    r["d_in"][4] += 4                        # misaligned input
    s.submit(r)
    c = s.progress()
    status = dict(zip(c["tag"].tolist(), c["status"].tolist()))
    assert status[0] == -2                   # length not a multiple of 8
    assert status[1] == -5                   # can never fit the arena / budget
    assert status[2] == 0                    # empty: done at once, nothing to release
    assert status[3] == -1                   # bad direction
    assert status[4] == -3                   # misaligned
    st = s.stats()
    assert st["rejected"] == 4 and st["queued"] == 0
    with pytest.raises(T.TdesError):
        s.release(0)


def test_arena_reuse_after_fragmentation():
    s = _server(arena_bytes=4 * 256, budget_bytes=1 << 20, slots=1, max_batch_msgs=4, test_polls=1)
    s.submit(_reqs([256] * 4))
    c = np.concatenate([s.progress(), s.progress()])
    assert len(c) == 4
    outs = sorted(c["d_out"].tolist())
    s.release(outs[1])
    s.release(outs[2])                       # frees a 512-byte hole in the middle
    s.submit(_reqs([512]))
    c2 = np.concatenate([s.progress(), s.progress()])
    assert c2["d_out"].tolist() == [outs[1]]


def test_bad_configs():
    with pytest.raises(T.TdesError):
        S.Server(FAKE_ARENA, 1 << 20, mode=S.HOST_TEST, slots=0)
    with pytest.raises(T.TdesError):
        S.Server(FAKE_ARENA + 8, 1 << 20, mode=S.HOST_TEST)
    with pytest.raises(T.TdesError):
        S.Server(FAKE_ARENA, 1 << 20, mode=9)


def test_open_loop_driver_in_host_mode():
    s = _server(arena_bytes=1 << 22, slots=2, max_batch_msgs=64, test_polls=2)
    n = 300
    reqs = _reqs(np.full(n, 64))
    arrival = np.linspace(0, 0.01, n)
    lat, status, wall, st = S.run_open_loop(s, reqs, arrival)
    assert (status == 0).all() and not np.isnan(lat).any()
    assert st["completed"] == n and st["released"] == n and st["in_flight_bytes"] == 0


def test_failed_launch_completes_its_requests_with_an_error():
    # A batch whose launch fails: its requests complete with
    # TDES_ERR_DEVICE and no result, their budget and arena space come back
    # at once, the slot is free again, and later batches run normally.
    s = _server(slots=1, max_batch_msgs=4, test_polls=2, test_fail_batch=2)
    s.submit(_reqs([512] * 4))
    s.progress()                              # batch 0 launched
    c0 = s.progress()                         # batch 0 done
    assert (c0["status"] == 0).all() and len(c0) == 4
    s.submit(_reqs([512] * 3, base=1 << 34))
    c1 = s.progress()                         # batch 1's launch fails
    assert len(c1) == 3
    assert (c1["status"] == -6).all() and (c1["d_out"] == 0).all() and (c1["batch"] == 1).all()
    assert b"injected launch failure" in T.lib().tdes_last_error()
    st = s.stats()
    assert st["failed"] == 3 and st["busy_slots"] == 0
    # only batch 0's outputs are still held
    assert st["in_flight_bytes"] == 4 * 512 and st["arena_used_bytes"] == 4 * 512
    with pytest.raises(T.TdesError):
        s.release(int(c1["d_out"][0]) or 1)
    for d in c0["d_out"]:
        s.release(d)
    s.submit(_reqs([512] * 2, base=1 << 35))
    s.progress()                              # batch 2 runs
    c2 = s.progress()
    assert len(c2) == 2 and (c2["status"] == 0).all() and (c2["batch"] == 2).all()
    for d in c2["d_out"]:
        s.release(d)
    st = s.stats()
    assert st["in_flight_bytes"] == 0 and st["arena_used_bytes"] == 0
    assert st["completed"] == 9 and st["failed"] == 3


def test_release_many():
    s = _server(slots=1, max_batch_msgs=8, test_polls=1)
    s.submit(_reqs([512] * 6))
    c = []
    for _ in range(5):
        c += list(s.progress())
        if len(c) == 6:
            break
    outs = [int(x["d_out"]) for x in c]
    assert s.release_many(outs[:3]) == 3
    st = s.stats()
    assert st["released"] == 3 and st["arena_used_bytes"] == 3 * 512
    # a stale entry among live ones: the live ones are still released and the
    # call reports the first bad entry
    with pytest.raises(T.TdesError) as e:
        s.release_many([outs[3], outs[0], outs[4], outs[5]])
    assert "entry 1" in str(e.value)
    st = s.stats()
    assert st["released"] == 6 and st["arena_used_bytes"] == 0 and st["in_flight_bytes"] == 0
    assert s.release_many([]) == 0
