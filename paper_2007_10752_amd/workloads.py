"""Seeded synthetic inputs for 3DES-ECB: keys, payloads, message layouts and
request traces.

This module draws random numbers and lays them out; it holds none of the
cipher's arithmetic, so both the GPU path's tests and the oracle take their
inputs from here.

The paper measured text files of 2^2 .. 2^17 64-bit blocks with unspecified
content and keys (Sec. V).  Payloads here are uniform random bytes (or the
structured all-zero / repeating-pattern buffers), keys are uniform random with
the DES parity bit (bit 8 of every byte) set for odd parity.
"""
import math

import numpy as np

SEED_BASE = 0x3DE50000  # data seed of workload i is SEED_BASE + i
KEY_SEED_OFFSET = 0x100
LAYOUT_SEED_OFFSET = 0x200

BLOCK = 8  # bytes per 64-bit block


def rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def odd_parity(keybytes):
    """Set the least significant bit of every byte so its popcount is odd."""
    k = np.array(keybytes, dtype=np.uint8).copy()
    hi = k & 0xFE
    ones = np.unpackbits(hi[:, None], axis=1).sum(axis=1)
    return (hi | ((ones + 1) & 1)).astype(np.uint8)


def key_bundle(gen, two_key=False):
    """24 key bytes K1||K2||K3; with two_key, K3 = K1."""
    k = odd_parity(gen.integers(0, 256, size=24, dtype=np.uint8))
    if two_key:
        k[16:24] = k[0:8]
    return k


def key_bundles(gen, n):
    """n independent 3-key bundles, shape (n, 24)."""
    raw = gen.integers(0, 256, size=(n, 24), dtype=np.uint8)
    return odd_parity(raw.reshape(-1)).reshape(n, 24)


def uniform_bytes(gen, nbytes):
    return gen.integers(0, 256, size=int(nbytes), dtype=np.uint8)


def pattern_bytes(nbytes, pattern=bytes(range(1, 9))):
    """Buffer made of one 8-byte pattern repeated."""
    p = np.frombuffer(bytes(pattern), dtype=np.uint8)
    assert p.size == BLOCK and nbytes % BLOCK == 0
    return np.tile(p, int(nbytes) // BLOCK)


# ---- batched workload: many messages, each with its own key and direction ----

def batched_layout(seed, n_msgs=16384, median=4096, sigma=1.0, lo=8, hi=1 << 20):
    """Message lengths log-normal (median ``median`` bytes, shape ``sigma``),
    clipped to [lo, hi] and rounded up to a multiple of 8; messages packed
    back to back.  Returns dict with offsets, lengths (bytes), key bundles
    (n, 24) and directions (0 encrypt, 1 decrypt)."""
    g = rng(seed)
    raw = g.lognormal(mean=math.log(median), sigma=sigma, size=n_msgs)
    lengths = np.clip(np.ceil(raw / BLOCK) * BLOCK, lo, hi).astype(np.int64)
    offsets = np.zeros(n_msgs, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)[:-1]
    keys = key_bundles(g, n_msgs)
    dirs = g.integers(0, 2, size=n_msgs).astype(np.uint32)
    return {"offsets": offsets, "lengths": lengths, "keys": keys, "dirs": dirs,
            "total": int(lengths.sum())}


# ---- serving workload: open-loop Poisson request trace ------------------------

SIZE_BANDS = ((0.70, 64, 1024), (0.25, 4096, 65536), (0.05, 1 << 20, 16 << 20))


def serving_trace(seed, rate, duration_s, bands=SIZE_BANDS):
    """Open-loop Poisson arrivals at ``rate`` requests/s over ``duration_s``.
    Sizes come from ``bands`` (probability, lo, hi), log-uniform within a band
    and rounded up to a multiple of 8.  Returns dict with arrival times (s),
    sizes (bytes), key bundles and directions."""
    g = rng(seed)
    n_est = int(rate * duration_s * 1.2) + 16
    gaps = g.exponential(1.0 / rate, size=n_est)
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        more = np.cumsum(g.exponential(1.0 / rate, size=n_est)) + t[-1]
        t = np.concatenate([t, more])
    t = t[t < duration_s]
    n = t.size
    probs = np.array([b[0] for b in bands])
    band = g.choice(len(bands), size=n, p=probs / probs.sum())
    lo = np.array([b[1] for b in bands], dtype=np.float64)[band]
    hi = np.array([b[2] for b in bands], dtype=np.float64)[band]
    u = g.random(n)
    size = np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))
    size = (np.ceil(size / BLOCK) * BLOCK).astype(np.int64)
    keys = key_bundles(g, n)
    dirs = g.integers(0, 2, size=n).astype(np.uint32)
    return {"arrival": t, "size": size, "keys": keys, "dirs": dirs}
