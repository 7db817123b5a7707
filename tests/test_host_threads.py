"""The library's host code called from several threads at once (no GPU
work): key schedules, kernel key material, argument errors with their
per-thread messages, and one request server per thread in its host test
mode.  ctypes releases the GIL around each foreign call, so the calls do run
concurrently; the sanitizer build (tests/test_sanitizers.py) runs this file
under ThreadSanitizer."""
import ctypes
import threading

import numpy as np

from paper_2007_10752_amd import serve as S
from paper_2007_10752_amd import tdes as T
from paper_2007_10752_amd import workloads as W

THREADS = 8
ITERS = 150


def _worker(i, key, want_rk, want_bs, want_sp, errors):
    lib = T.lib()
    try:
        for it in range(ITERS):
            sched = T.key_schedule(key)
            assert sched.round_keys() == want_rk
            assert T.kernel_key_bytes(sched, it % 2, T.KERNELS["bitslice"]) == want_bs[it % 2]
            assert T.kernel_key_bytes(sched, it % 2, T.KERNELS["spbox"]) == want_sp[it % 2]
            # an argument error naming this thread's own length: the message is
            # per thread and must not be overwritten by the other threads
            n = 8 * (1000 * i + it) + 1 + (it % 7)
            st = lib.tdes_ecb_crypt(ctypes.byref(sched), 0, 0, ctypes.c_void_p(0x1000),
                                    ctypes.c_void_p(0x100000), n, None)
            assert st == -2, st
            assert ("length %d " % n) in lib.tdes_last_error().decode(), \
                lib.tdes_last_error().decode()
        # a request server of this thread's own, in host test mode
        srv = S.Server(1 << 40, 1 << 20, mode=S.HOST_TEST, slots=3, max_batch_msgs=5,
                       test_polls=2, budget_bytes=64 << 10)
        n = 200
        r = np.zeros(n, dtype=S.REQUEST)
        r["d_in"] = (1 << 30) + np.arange(n, dtype=np.uint64) * np.uint64(1 << 20)
        r["nbytes"] = 8 * (1 + (np.arange(n) * 37 + i) % 512)
        r["dir"] = np.arange(n) % 2
        r["tag"] = np.arange(n)
        srv.submit(r)
        tags = []
        for _ in range(10000):
            c = srv.progress()
            assert (c["status"] == 0).all()
            tags += c["tag"].tolist()
            for d in c["d_out"]:
                srv.release(d)
            if len(tags) == n:
                break
        assert tags == list(range(n))
        st = srv.stats()
        assert st["in_flight_bytes"] == 0 and st["arena_used_bytes"] == 0
        srv.close()
    except BaseException as e:  # reported by the main thread
        errors.append((i, repr(e)))


def test_concurrent_host_calls():
    keys = [W.key_bundle(W.rng(W.SEED_BASE + 0xC00 + i)) for i in range(THREADS)]
    want = []
    for k in keys:
        s = T.key_schedule(k)
        want.append((s.round_keys(),
                     [T.kernel_key_bytes(s, d, T.KERNELS["bitslice"]) for d in (0, 1)],
                     [T.kernel_key_bytes(s, d, T.KERNELS["spbox"]) for d in (0, 1)]))
    errors = []
    ts = [threading.Thread(target=_worker, args=(i, keys[i]) + want[i] + (errors,))
          for i in range(THREADS)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors
