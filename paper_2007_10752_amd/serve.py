"""ctypes binding of the request server (include/tdes_serve.h) and an
open-loop load driver for it.

The driver replays a request trace (arrival times, sizes, key bundles,
directions; see workloads.serving_trace) against a server: every request is
submitted at its scheduled arrival time whatever the state of earlier ones,
and its latency is measured from that scheduled time to the completion the
server reports, so a backlog shows up as latency rather than as a slower
arrival rate.  Payloads are slices of a device-resident pool.
"""
import ctypes

import numpy as np

from . import tdes

BATCHED, PLAIN, HOST_TEST = 0, 1, 2


class ServerConfig(ctypes.Structure):
    _fields_ = [("d_arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_uint64), ("mode", ctypes.c_uint32),
                ("slots", ctypes.c_uint32), ("max_batch_msgs", ctypes.c_uint32),
                ("test_polls", ctypes.c_uint32), ("max_batch_bytes", ctypes.c_uint64),
                ("test_fail_batch", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "submitted", "admitted", "completed", "released", "rejected", "queued",
        "in_flight_bytes", "peak_in_flight_bytes", "arena_used_bytes", "peak_arena_used_bytes",
        "batches", "batched_msgs", "batched_bytes")] + [
        ("busy_slots", ctypes.c_uint32), ("peak_busy_slots", ctypes.c_uint32),
        ("failed", ctypes.c_uint64)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


# numpy layouts of tdes_request (56 bytes) and tdes_completion (64 bytes)
REQUEST = np.dtype([("key24", np.uint8, 24), ("dir", "<u4"), ("reserved", "<u4"),
                    ("d_in", "<u8"), ("nbytes", "<u8"), ("tag", "<u8")])
COMPLETION = np.dtype([("tag", "<u8"), ("d_out", "<u8"), ("nbytes", "<u8"), ("status", "<i4"),
                       ("batch", "<u4"), ("t_submit", "<f8"), ("t_admit", "<f8"),
                       ("t_launch", "<f8"), ("t_done", "<f8")])
assert REQUEST.itemsize == 56 and COMPLETION.itemsize == 64

_bound = False


def _lib():
    global _bound
    L = tdes.lib()
    if not _bound:
        vp = ctypes.c_void_p
        L.tdes_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
        L.tdes_server_create.restype = ctypes.c_int
        L.tdes_server_destroy.argtypes = [vp]
        L.tdes_server_destroy.restype = None
        L.tdes_server_submit.argtypes = [vp, vp, ctypes.c_size_t]
        L.tdes_server_submit.restype = ctypes.c_int
        L.tdes_server_progress.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.tdes_server_progress.restype = ctypes.c_int
        L.tdes_server_release.argtypes = [vp, vp]
        L.tdes_server_release.restype = ctypes.c_int
        L.tdes_server_release_many.argtypes = [vp, vp, ctypes.c_size_t,
                                               ctypes.POINTER(ctypes.c_size_t)]
        L.tdes_server_release_many.restype = ctypes.c_int
        L.tdes_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.tdes_server_get_stats.restype = ctypes.c_int
        L.tdes_server_now.argtypes = []
        L.tdes_server_now.restype = ctypes.c_double
        _bound = True
    return L


def now():
    return _lib().tdes_server_now()


class Server:
    """One tdes_server.  ``arena_ptr`` is a device address the caller owns
    (a fake, never-dereferenced address is fine in HOST_TEST mode)."""

    def __init__(self, arena_ptr, arena_bytes, budget_bytes=0, mode=BATCHED, slots=4,
                 max_batch_msgs=4096, max_batch_bytes=0, test_polls=2, completion_cap=65536,
                 test_fail_batch=0):
        self.h = None
        L = _lib()
        cfg = ServerConfig(arena_ptr, arena_bytes, budget_bytes, mode, slots, max_batch_msgs,
                           test_polls, max_batch_bytes, test_fail_batch, 0)
        h = ctypes.c_void_p()
        tdes._check(L.tdes_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self.arena_ptr = arena_ptr
        self._buf = np.zeros(completion_cap, dtype=COMPLETION)
        self._n = ctypes.c_size_t()

    def close(self):
        if self.h:
            _lib().tdes_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def submit(self, reqs):
        """Submit a numpy array of REQUEST records."""
        reqs = np.ascontiguousarray(reqs, dtype=REQUEST)
        tdes._check(_lib().tdes_server_submit(self.h, reqs.ctypes.data, len(reqs)))

    def progress(self):
        """One progress step; returns a numpy array of COMPLETION records."""
        tdes._check(_lib().tdes_server_progress(self.h, self._buf.ctypes.data, len(self._buf),
                                                ctypes.byref(self._n)))
        return self._buf[: self._n.value].copy()

    def release(self, d_out):
        tdes._check(_lib().tdes_server_release(self.h, ctypes.c_void_p(int(d_out))))

    def release_many(self, d_outs):
        """Release many results at once (array-like of device addresses);
        returns how many were released."""
        a = np.ascontiguousarray(d_outs, dtype=np.uint64)
        k = ctypes.c_size_t()
        tdes._check(_lib().tdes_server_release_many(self.h, a.ctypes.data, len(a), ctypes.byref(k)))
        return k.value

    def stats(self):
        st = ServerStats()
        tdes._check(_lib().tdes_server_get_stats(self.h, ctypes.byref(st)))
        return st.as_dict()


def make_requests(trace, pool_ptr, pool_bytes, seed):
    """REQUEST records for a trace, payloads at seeded 8-byte aligned offsets
    of a device pool."""
    n = len(trace["size"])
    g = np.random.Generator(np.random.PCG64(seed))
    room = np.maximum(pool_bytes - trace["size"], 0) // 8
    offs = (g.integers(0, np.iinfo(np.int64).max, size=n) % (room + 1)) * 8
    r = np.zeros(n, dtype=REQUEST)
    r["key24"] = trace["keys"]
    r["dir"] = trace["dirs"]
    r["d_in"] = np.uint64(pool_ptr) + offs.astype(np.uint64)
    r["nbytes"] = trace["size"]
    r["tag"] = np.arange(n, dtype=np.uint64)
    return r


def run_open_loop(server, reqs, arrival, on_complete=None, timeout_s=60.0):
    """Replay requests at their scheduled arrival times (seconds from start).
    Requests are tagged with their position in ``reqs`` (the completions
    handed to on_complete carry that position as their tag).  Returns
    per-request latency (scheduled arrival -> completion seen), status, the
    wall time from start to the last completion, and the server's stats."""
    n = len(reqs)
    reqs = np.array(reqs, dtype=REQUEST, copy=True)
    reqs["tag"] = np.arange(n, dtype=np.uint64)
    lat = np.full(n, np.nan)
    status = np.zeros(n, dtype=np.int32)
    done = 0
    nxt = 0
    t0 = now()
    while done < n:
        t = now() - t0
        if t > timeout_s:
            raise TimeoutError("open-loop run did not finish in %.0f s" % timeout_s)
        k = int(np.searchsorted(arrival, t, side="right"))
        if k > nxt:
            server.submit(reqs[nxt:k])
            nxt = k
        comp = server.progress()
        if len(comp):
            tags = comp["tag"].astype(np.int64)
            lat[tags] = comp["t_done"] - (t0 + arrival[tags])
            status[tags] = comp["status"]
            if on_complete is not None:
                on_complete(comp)
            live = comp["d_out"][(comp["status"] == 0) & (comp["nbytes"] > 0)]
            if len(live):
                server.release_many(live)
            done += len(comp)
    wall = now() - t0
    return lat, status, wall, server.stats()


# request size bands for the latency breakdown: up to 1 KiB, up to 64 KiB, larger
BANDS = (("small", 0, 1024), ("medium", 1025, 65536), ("large", 65537, 1 << 62))


def summarize(lat, sizes, wall, stats, rate, duration):
    ok = lat[~np.isnan(lat)]
    by_band = {}
    for name, lo, hi in BANDS:
        sel = (sizes >= lo) & (sizes <= hi) & ~np.isnan(lat)
        if sel.any():
            by_band[name] = {"n": int(sel.sum()),
                             "p50_ms": round(float(np.percentile(lat[sel], 50)) * 1e3, 4),
                             "p99_ms": round(float(np.percentile(lat[sel], 99)) * 1e3, 4)}
    return {"rate_req_s": rate, "duration_s": duration, "requests": int(len(lat)),
            "p50_ms": round(float(np.percentile(ok, 50)) * 1e3, 4),
            "p99_ms": round(float(np.percentile(ok, 99)) * 1e3, 4),
            "by_size": by_band,
            "GBps": round(float(np.sum(sizes)) / wall / 1e9, 4),
            "offered_GBps": round(float(np.sum(sizes)) / duration / 1e9, 4),
            "batches": stats["batches"],
            "mean_batch": round(stats["batched_msgs"] / max(1, stats["batches"]), 2),
            "peak_in_flight_MiB": round(stats["peak_in_flight_bytes"] / 2**20, 2),
            "peak_busy_slots": stats["peak_busy_slots"]}
