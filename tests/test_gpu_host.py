"""GPU parity of the host-resident form (tdes_ecb_host): host buffers in,
host buffers out.  Two modes: direct (the kernel works on pinned host memory
over PCIe) and staged (chunks through device slots on several streams).
Every result is compared bit for bit with the oracle.  The cases are:

* ragged sizes around chunk and wave-chunk boundaries, and chunks off the
  16-byte grid;
* one slot (no overlap) and more slots than the library uses;
* pinned and pageable memory, in place;
* the 64 MiB case in full, in both directions and both modes;
* direct mode refusing pageable memory and a range past its allocation."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2007_10752_amd import tdes as T
from paper_2007_10752_amd import workloads as W

pytestmark = pytest.mark.gpu

CHUNK = 64 * 1024


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pinned(torch, host):
    t = torch.empty(host.size, dtype=torch.uint8, pin_memory=True)
    t.numpy()[:] = host
    return t


@pytest.mark.parametrize("nbytes", [8, CHUNK - 8, CHUNK, CHUNK + 8, 3 * CHUNK + 24, 7 * CHUNK + 4096])
@pytest.mark.parametrize("n_slots", [1, 3, 12])
def test_ragged_sizes_and_slot_counts(torch_dev, nbytes, n_slots):
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x500 + nbytes % 1000 + n_slots)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, nbytes)
    pipe = T.HostPipeline(CHUNK, n_slots)
    _say("host path", nbytes, "bytes,", n_slots, "slots")
    got = pipe.run(key, _pinned(torch, data))
    assert np.array_equal(got.numpy(), oracle.tdes_ecb(key, data))
    back = pipe.run(key, got, decrypt=True)
    assert np.array_equal(back.numpy(), data)


def test_chunks_off_the_16_byte_grid(torch_dev):
    # 8,008-byte chunks: every other slot starts 8 bytes off a 16-byte
    # boundary (the kernel's 8-byte path), many chunks per slot, a short last one.
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x515)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 8008 * 37 + 8 * 5)
    pipe = T.HostPipeline(8008, 3)
    _say("host path 8008-byte chunks")
    got = pipe.run(key, _pinned(torch, data), decrypt=True)
    assert np.array_equal(got.numpy(), oracle.tdes_ecb(key, data, decrypt=True))


def test_pageable_and_in_place(torch_dev):
    g = W.rng(W.SEED_BASE + 0x510)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, 5 * CHUNK + 8 * 13)
    pipe = T.HostPipeline(CHUNK, 4)
    _say("host path pageable")
    got = pipe.run(key, data.copy())  # numpy: pageable memory
    want = oracle.tdes_ecb(key, data)
    assert np.array_equal(got, want)
    buf = data.copy()
    assert pipe.run(key, buf, buf) is buf  # in place
    assert np.array_equal(buf, want)
    dec = oracle.tdes_ecb(key, data, decrypt=True)
    assert np.array_equal(pipe.run(key, data, decrypt=True), dec)


def test_empty_is_noop(torch_dev):
    pipe = T.HostPipeline(CHUNK, 2)
    out = pipe.run(bytes(24), np.zeros(0, np.uint8))
    assert out.size == 0


@pytest.mark.parametrize("decrypt", [False, True])
def test_64mib_full(torch_dev, decrypt):
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 1)
    data = W.uniform_bytes(g, 8 * 8388608)
    key = W.key_bundle(W.rng(W.SEED_BASE + 1 + W.KEY_SEED_OFFSET))
    pipe = T.HostPipeline(4 << 20, 4)
    _say("host path 64MiB decrypt", decrypt)
    h_in = _pinned(torch, data)
    want = oracle.tdes_ecb(key, data, decrypt)
    got = pipe.run(key, h_in, decrypt=decrypt)
    assert np.array_equal(got.numpy(), want)
    direct = T.ecb_host(key, h_in, decrypt=decrypt)
    assert np.array_equal(direct.numpy(), want)
    # and the same bytes as the device path
    x = h_in.cuda()
    dev = T.ecb(key, x, decrypt=decrypt)
    assert np.array_equal(got.numpy(), dev.cpu().numpy())


@pytest.mark.parametrize("nbytes", [8, 16384 - 8, 16384, 16384 + 8, 3 * 16384 + 24, (1 << 20) + 8])
def test_direct_ragged_and_in_place(torch_dev, nbytes):
    torch = torch_dev
    g = W.rng(W.SEED_BASE + 0x520 + nbytes % 1000)
    key = W.key_bundle(g)
    data = W.uniform_bytes(g, nbytes)
    _say("host direct", nbytes)
    h = _pinned(torch, data)
    want = oracle.tdes_ecb(key, data)
    got = T.ecb_host(key, h)
    assert got.is_pinned()
    assert np.array_equal(got.numpy(), want)
    assert np.array_equal(T.ecb_host(key, got, decrypt=True).numpy(), data)
    assert T.ecb_host(key, h, h) is h  # in place
    assert np.array_equal(h.numpy(), want)


def _allocation_extent(ptr):
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemGetAddressRange.argtypes = [ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_size_t), ctypes.c_void_p]
    hip.hipMemGetAddressRange.restype = ctypes.c_int
    base, size = ctypes.c_void_p(), ctypes.c_size_t()
    rc = hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), ctypes.c_void_p(ptr))
    return rc, base.value or 0, size.value


def test_direct_refuses_unmapped_ranges(torch_dev):
    torch = torch_dev
    key = W.key_bundle(W.rng(W.SEED_BASE + 0x530))
    data = W.uniform_bytes(W.rng(W.SEED_BASE + 0x531), 64 * 1024)
    _say("host direct refusals")
    with pytest.raises(T.TdesError) as e:
        T.ecb_host(key, data.copy())  # pageable numpy memory
    assert e.value.status == -1
    # A range running past the pinned allocation that holds its start.  The
    # extent the library checks against is read first: only a sane one (the
    # buffer, well under 1 TiB) lets the call below go ahead.
    h = _pinned(torch, data)
    rc, base, size = _allocation_extent(h.data_ptr())
    assert rc == 0 and base <= h.data_ptr() and h.data_ptr() + h.numel() <= base + size < base + (1 << 40)
    with pytest.raises(T.TdesError) as e:
        T.ecb_host_ptr(T.key_schedule(key), T.ENCRYPT, h.data_ptr(), h.data_ptr(), 1 << 40,
                       None, 0, 0)
    assert e.value.status == -1
    assert np.array_equal(h.numpy(), data)  # untouched
    # the refusals leave no HIP error behind for the next call to report
    assert torch.zeros(8, device="cuda").sum().item() == 0
