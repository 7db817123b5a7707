"""ctypes binding of libtdes.so (C ABI in include/tdes.h).

Argument marshalling only: key bytes and schedules are passed through,
tensors are turned into device pointers and streams into hipStream_t
handles.  Every step of the cipher runs in the library's HIP kernels; there
is no CPU fallback, and a missing library is an error.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# TDES_LIB names another build of the same library (for comparing builds).
LIB_PATH = os.environ.get("TDES_LIB") or os.path.join(PKG, "libtdes.so")

ENCRYPT, DECRYPT = 0, 1
KERNEL_AUTO, KERNEL_BITSLICE, KERNEL_SPBOX = 0, 1, 2
KERNELS = {"auto": KERNEL_AUTO, "bitslice": KERNEL_BITSLICE, "spbox": KERNEL_SPBOX}

STATUS = {0: "TDES_OK", -1: "TDES_ERR_ARG", -2: "TDES_ERR_LENGTH", -3: "TDES_ERR_ALIGN",
          -4: "TDES_ERR_OVERLAP", -5: "TDES_ERR_NOMEM", -6: "TDES_ERR_DEVICE"}

# Exported symbols, checked against include/*.h by the tests.
SYMBOLS = ("tdes_key_schedule", "tdes_ecb_encrypt", "tdes_ecb_decrypt", "tdes_ecb_crypt",
           "tdes_last_error", "tdes_abi_version", "tdes_kernel_key_bytes", "tdes_probe_valu",
           "tdes_probe_copy", "tdes_probe_lds", "tdes_schedule_upload", "tdes_schedule_expand",
           "tdes_batch_workspace_bytes", "tdes_batch_submit", "tdes_batch_submit_noalloc",
           "tdes_server_create",
           "tdes_server_destroy", "tdes_server_submit", "tdes_server_progress",
           "tdes_server_release", "tdes_server_release_many", "tdes_server_get_stats",
           "tdes_server_now", "tdes_ecb_host",
           "tdes_ctr_crypt", "tdes_cbc_decrypt", "tdes_ecb_paper_design",
           "tdes_batch_autotune", "tdes_batch_autotune_streams", "tdes_batch_get_config",
           "tdes_ecb_auto_kernel",
           "tdes_batch_set_config", "tdes_batch_config_load", "tdes_batch_config_save")

DEVICE_SCHEDULE_BYTES = 800
MSG_BYTES = 32


class TdesError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, message))
        self.status = status


class Schedule(ctypes.Structure):
    """tdes_schedule: k[b][i] = round key i+1 of base key b+1 (48 bits)."""
    _fields_ = [("k", (ctypes.c_uint64 * 16) * 3)]

    def round_keys(self):
        return [[int(self.k[b][i]) for i in range(16)] for b in range(3)]


_lib = None


class BatchConfig(ctypes.Structure):
    """tdes_batch_config: the batched kernel's variant and grid."""
    _fields_ = [("kmax", ctypes.c_uint32), ("waves", ctypes.c_uint32),
                ("grid_mult", ctypes.c_uint32), ("saved", ctypes.c_uint32)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("%s is missing: build it with `python -m paper_2007_10752_amd.build`"
                               % LIB_PATH)
        # torch ships its own HIP runtime under the same soname as the
        # system's.  Whichever is loaded first serves the whole process;
        # loading torch first makes it the one torch was built against, so
        # the library and torch's tensors share one runtime (the other order
        # left the library without a device).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        sched_p = ctypes.POINTER(Schedule)
        L.tdes_key_schedule.argtypes = [ctypes.POINTER(ctypes.c_uint8), sched_p]
        L.tdes_key_schedule.restype = ctypes.c_int
        for name in ("tdes_ecb_encrypt", "tdes_ecb_decrypt"):
            fn = getattr(L, name)
            fn.argtypes = [sched_p, vp, vp, sz, vp]
            fn.restype = ctypes.c_int
        L.tdes_ecb_crypt.argtypes = [sched_p, ctypes.c_int, ctypes.c_int, vp, vp, sz, vp]
        L.tdes_ecb_crypt.restype = ctypes.c_int
        L.tdes_last_error.argtypes = []
        L.tdes_last_error.restype = ctypes.c_char_p
        L.tdes_abi_version.argtypes = []
        L.tdes_abi_version.restype = ctypes.c_int
        L.tdes_schedule_upload.argtypes = [sched_p, sz, vp, vp]
        L.tdes_schedule_upload.restype = ctypes.c_int
        L.tdes_schedule_expand.argtypes = [vp, sz, vp, vp]
        L.tdes_schedule_expand.restype = ctypes.c_int
        L.tdes_batch_workspace_bytes.argtypes = [sz]
        L.tdes_batch_workspace_bytes.restype = sz
        L.tdes_batch_submit.argtypes = [vp, sz, vp, sz, vp, sz, vp, sz, vp, sz, vp]
        L.tdes_batch_submit.restype = ctypes.c_int
        L.tdes_batch_submit_noalloc.argtypes = [vp, sz, vp, sz, vp, sz, vp, sz, vp, vp]
        L.tdes_batch_submit_noalloc.restype = ctypes.c_int
        cfg_p = ctypes.POINTER(BatchConfig)
        L.tdes_batch_autotune.argtypes = [vp, sz, vp, sz, vp, sz, vp, sz, vp, sz, vp,
                                          ctypes.c_int, cfg_p]
        L.tdes_batch_autotune.restype = ctypes.c_int
        vpp = ctypes.POINTER(ctypes.c_void_p)
        L.tdes_batch_autotune_streams.argtypes = [vp, sz, vp, sz, vp, sz, vpp, sz, vpp, sz, vpp,
                                                  ctypes.c_int, ctypes.c_int, cfg_p]
        L.tdes_batch_autotune_streams.restype = ctypes.c_int
        L.tdes_ecb_auto_kernel.argtypes = [sz]
        L.tdes_ecb_auto_kernel.restype = ctypes.c_int
        L.tdes_batch_get_config.argtypes = [cfg_p]
        L.tdes_batch_get_config.restype = ctypes.c_int
        L.tdes_batch_set_config.argtypes = [cfg_p]
        L.tdes_batch_set_config.restype = ctypes.c_int
        L.tdes_batch_config_load.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_uint32,
                                             cfg_p]
        L.tdes_batch_config_load.restype = ctypes.c_int
        L.tdes_batch_config_save.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_uint32,
                                             cfg_p, ctypes.c_double]
        L.tdes_batch_config_save.restype = ctypes.c_int
        L.tdes_ctr_crypt.argtypes = [sched_p, ctypes.POINTER(ctypes.c_uint8), vp, vp, sz, vp]
        L.tdes_ctr_crypt.restype = ctypes.c_int
        L.tdes_cbc_decrypt.argtypes = [sched_p, ctypes.POINTER(ctypes.c_uint8), vp, vp, sz, vp]
        L.tdes_cbc_decrypt.restype = ctypes.c_int
        L.tdes_ecb_paper_design.argtypes = [sched_p, ctypes.c_int, vp, vp, sz, vp]
        L.tdes_ecb_paper_design.restype = ctypes.c_int
        L.tdes_ecb_host.argtypes = [sched_p, ctypes.c_int, vp, vp, sz, vp, sz, sz]
        L.tdes_ecb_host.restype = ctypes.c_int
        L.tdes_kernel_key_bytes.argtypes = [sched_p, ctypes.c_int, ctypes.c_int, vp, sz]
        L.tdes_kernel_key_bytes.restype = ctypes.c_long
        L.tdes_probe_valu.argtypes = [ctypes.c_int, vp, ctypes.c_uint, ctypes.c_uint, vp]
        L.tdes_probe_valu.restype = ctypes.c_int
        L.tdes_probe_lds.argtypes = [ctypes.c_int, vp, ctypes.c_uint, ctypes.c_uint, vp]
        L.tdes_probe_lds.restype = ctypes.c_int
        L.tdes_probe_copy.argtypes = [vp, vp, sz, vp]
        L.tdes_probe_copy.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise TdesError(status, lib().tdes_last_error().decode(errors="replace"))


def key_schedule(key24):
    """tdes_key_schedule on a 24-byte key bundle K1||K2||K3."""
    kb = bytes(bytearray(key24))
    if len(kb) != 24:
        raise ValueError("key bundle must be 24 bytes")
    buf = (ctypes.c_uint8 * 24).from_buffer_copy(kb)
    s = Schedule()
    _check(lib().tdes_key_schedule(buf, ctypes.byref(s)))
    return s


def ecb_crypt_ptr(schedule, direction, kernel, d_in, d_out, nbytes, stream=0):
    """tdes_ecb_crypt on raw device addresses (ints) and a hipStream_t (int)."""
    _check(lib().tdes_ecb_crypt(ctypes.byref(schedule), int(direction), int(kernel),
                                ctypes.c_void_p(d_in), ctypes.c_void_p(d_out),
                                ctypes.c_size_t(nbytes), ctypes.c_void_p(stream)))


def auto_kernel(nbytes):
    """The kernel TDES_KERNEL_AUTO runs for nbytes on the current device, by
    name ("spbox" or "bitslice")."""
    k = lib().tdes_ecb_auto_kernel(int(nbytes))
    if k < 0:
        raise TdesError(k, lib().tdes_last_error().decode())
    return {KERNEL_BITSLICE: "bitslice", KERNEL_SPBOX: "spbox"}[k]


def kernel_key_bytes(schedule, direction, kernel):
    """The kernel argument a launch would receive (tdes_kernel_key_bytes)."""
    buf = ctypes.create_string_buffer(4096)
    n = lib().tdes_kernel_key_bytes(ctypes.byref(schedule), int(direction), int(kernel), buf, 4096)
    if n < 0:
        _check(int(n))
    return buf.raw[:n]


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _schedule(key):
    return key if isinstance(key, Schedule) else key_schedule(key)


def ecb(key, x, out=None, decrypt=False, kernel="auto", stream=None):
    """3DES-EDE ECB over a contiguous uint8 CUDA tensor (length a multiple of
    8).  ``key`` is a 24-byte bundle or a Schedule; ``out`` may be ``x``
    (in place) or a new tensor is allocated.  Enqueued on ``stream`` (default:
    torch's current stream)."""
    import torch
    if not (x.is_cuda and x.dtype == torch.uint8 and x.is_contiguous()):
        raise ValueError("x must be a contiguous uint8 CUDA tensor")
    if out is None:
        out = torch.empty_like(x)
    if not (out.is_cuda and out.dtype == torch.uint8 and out.is_contiguous()
            and out.numel() == x.numel()):
        raise ValueError("out must be a contiguous uint8 CUDA tensor shaped like x")
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    ecb_crypt_ptr(_schedule(key), DECRYPT if decrypt else ENCRYPT, k,
                  x.data_ptr(), out.data_ptr(), x.numel(), _stream_handle(stream))
    return out


def encrypt(key, x, out=None, kernel="auto", stream=None):
    return ecb(key, x, out, False, kernel, stream)


def ctr_crypt_ptr(schedule, iv8, d_in, d_out, nbytes, stream=0):
    iv = (ctypes.c_uint8 * 8).from_buffer_copy(bytes(bytearray(iv8)))
    _check(lib().tdes_ctr_crypt(ctypes.byref(schedule), iv, ctypes.c_void_p(d_in),
                                ctypes.c_void_p(d_out), ctypes.c_size_t(nbytes),
                                ctypes.c_void_p(stream)))


def ctr(key, iv8, x, out=None, stream=None):
    """3DES-EDE in counter mode over a contiguous uint8 CUDA tensor: out =
    x XOR E(counter blocks IV, IV + 1, ...), the 8-byte IV read as a
    big-endian integer.  Its own inverse.  ``out`` may be ``x``."""
    import torch
    if not (x.is_cuda and x.dtype == torch.uint8 and x.is_contiguous()):
        raise ValueError("x must be a contiguous uint8 CUDA tensor")
    if out is None:
        out = torch.empty_like(x)
    if not (out.is_cuda and out.dtype == torch.uint8 and out.is_contiguous()
            and out.numel() == x.numel()):
        raise ValueError("out must be a contiguous uint8 CUDA tensor shaped like x")
    if len(bytes(bytearray(iv8))) != 8:
        raise ValueError("iv must be 8 bytes")
    ctr_crypt_ptr(_schedule(key), iv8, x.data_ptr(), out.data_ptr(), x.numel(),
                  _stream_handle(stream))
    return out


def cbc_decrypt_ptr(schedule, iv8, d_in, d_out, nbytes, stream=0):
    iv = (ctypes.c_uint8 * 8).from_buffer_copy(bytes(bytearray(iv8)))
    _check(lib().tdes_cbc_decrypt(ctypes.byref(schedule), iv, ctypes.c_void_p(d_in),
                                  ctypes.c_void_p(d_out), ctypes.c_size_t(nbytes),
                                  ctypes.c_void_p(stream)))


def cbc_decrypt(key, iv8, x, out=None, stream=None):
    """3DES-EDE CBC decryption of a contiguous uint8 CUDA tensor: out block i
    = D(x block i) XOR x block i - 1 (the 8-byte IV before the first).
    ``out`` must not overlap ``x``."""
    import torch
    if not (x.is_cuda and x.dtype == torch.uint8 and x.is_contiguous()):
        raise ValueError("x must be a contiguous uint8 CUDA tensor")
    if out is None:
        out = torch.empty_like(x)
    if not (out.is_cuda and out.dtype == torch.uint8 and out.is_contiguous()
            and out.numel() == x.numel()):
        raise ValueError("out must be a contiguous uint8 CUDA tensor shaped like x")
    if len(bytes(bytearray(iv8))) != 8:
        raise ValueError("iv must be 8 bytes")
    cbc_decrypt_ptr(_schedule(key), iv8, x.data_ptr(), out.data_ptr(), x.numel(),
                    _stream_handle(stream))
    return out


def paper_design_ptr(schedule, direction, d_in, d_out, nbytes, stream=0):
    """The paper's one-thread-per-bit design (comparison only)."""
    _check(lib().tdes_ecb_paper_design(ctypes.byref(schedule), direction, ctypes.c_void_p(d_in),
                                       ctypes.c_void_p(d_out), ctypes.c_size_t(nbytes),
                                       ctypes.c_void_p(stream)))


HOST_MAX_SLOTS = 8


def ecb_host_ptr(schedule, direction, h_in, h_out, nbytes, d_work, work_bytes, chunk_bytes):
    _check(lib().tdes_ecb_host(ctypes.byref(schedule), direction, ctypes.c_void_p(h_in),
                               ctypes.c_void_p(h_out), ctypes.c_size_t(nbytes),
                               ctypes.c_void_p(d_work), ctypes.c_size_t(work_bytes),
                               ctypes.c_size_t(chunk_bytes)))


def _host_ptr(a):
    """Address and size of a contiguous host byte buffer: a numpy uint8 array
    or a CPU uint8 torch tensor (pinned or not)."""
    import numpy as np
    if isinstance(a, np.ndarray):
        if a.dtype != np.uint8 or not a.flags["C_CONTIGUOUS"]:
            raise ValueError("host buffer must be a contiguous uint8 array")
        return a.ctypes.data, a.size
    import torch
    if a.is_cuda or a.dtype != torch.uint8 or not a.is_contiguous():
        raise ValueError("host buffer must be a contiguous uint8 CPU tensor")
    return a.data_ptr(), a.numel()


def _host_out(h_in, h_out):
    import torch
    if h_out is None:
        h_out = (h_in.copy() if hasattr(h_in, "flags") else
                 torch.empty(h_in.shape, dtype=torch.uint8, pin_memory=h_in.is_pinned()))
    a, n = _host_ptr(h_in)
    b, m = _host_ptr(h_out)
    if m != n:
        raise ValueError("h_out must have the size of h_in")
    return h_out, a, b, n


def ecb_host(key, h_in, h_out=None, decrypt=False):
    """Direct host-resident 3DES-EDE ECB: the kernel reads h_in and writes
    h_out (pinned CPU uint8 tensors; h_out a new pinned tensor if None, h_in
    for in place) in host memory over PCIe.  Returns h_out once it holds the
    result."""
    import torch
    h_out, a, b, n = _host_out(h_in, h_out)
    # the library's stream does not wait for torch's (pending copies into h_in)
    torch.cuda.current_stream().synchronize()
    ecb_host_ptr(_schedule(key), DECRYPT if decrypt else ENCRYPT, a, b, n, None, 0, 0)
    return h_out


class HostPipeline:
    """Staged host-resident 3DES-EDE ECB (any host memory): n_slots device
    slots of chunk_bytes in one torch tensor, reused by every run."""

    def __init__(self, chunk_bytes=8 << 20, n_slots=4):
        import torch
        self.chunk_bytes = int(chunk_bytes)
        self.work = torch.empty(self.chunk_bytes * int(n_slots), dtype=torch.uint8, device="cuda")

    def run(self, key, h_in, h_out=None, decrypt=False):
        """3DES-EDE ECB of host buffer h_in into h_out (same type; a new
        buffer like h_in if None; h_in itself for in place).  Returns h_out
        once it holds the result."""
        import torch
        h_out, a, b, n = _host_out(h_in, h_out)
        # the library's streams do not wait for torch's: let pending work on
        # the workspace finish first
        torch.cuda.current_stream().synchronize()
        ecb_host_ptr(_schedule(key), DECRYPT if decrypt else ENCRYPT, a, b, n,
                     self.work.data_ptr(), self.work.numel(), self.chunk_bytes)
        return h_out


def decrypt(key, x, out=None, kernel="auto", stream=None):
    return ecb(key, x, out, True, kernel, stream)


# ---- batched form -----------------------------------------------------------

def key_schedules(keys):
    """Schedules of many 24-byte bundles (array-like of shape (n, 24)), as a
    ctypes array of tdes_schedule."""
    import numpy as np
    k = np.ascontiguousarray(keys, dtype=np.uint8).reshape(-1, 24)
    arr = (Schedule * len(k))()
    buf = (ctypes.c_uint8 * 24)()
    L = lib()
    for i in range(len(k)):
        ctypes.memmove(buf, k[i].ctypes.data, 24)
        _check(L.tdes_key_schedule(buf, ctypes.byref(arr[i])))
    return arr


def schedule_upload(schedules, d_dst, stream=0):
    """tdes_schedule_upload of a ctypes array of Schedule to device address d_dst."""
    _check(lib().tdes_schedule_upload(schedules, len(schedules), ctypes.c_void_p(d_dst),
                                      ctypes.c_void_p(stream)))


def schedule_expand(d_keys24, n, d_schedules, stream=0):
    """tdes_schedule_expand: n 24-byte bundles (device) -> device schedules."""
    _check(lib().tdes_schedule_expand(ctypes.c_void_p(d_keys24), n, ctypes.c_void_p(d_schedules),
                                      ctypes.c_void_p(stream)))


def batch_workspace_bytes(n_msgs):
    return int(lib().tdes_batch_workspace_bytes(n_msgs))


def batch_submit_ptr(d_msgs, n_msgs, d_sched, n_sched, d_in, in_bytes, d_out, out_bytes, d_ws,
                     ws_bytes, stream=0):
    """tdes_batch_submit on raw device addresses."""
    _check(lib().tdes_batch_submit(ctypes.c_void_p(d_msgs), n_msgs, ctypes.c_void_p(d_sched),
                                   n_sched, ctypes.c_void_p(d_in), in_bytes,
                                   ctypes.c_void_p(d_out), out_bytes, ctypes.c_void_p(d_ws),
                                   ws_bytes, ctypes.c_void_p(stream)))


# Most messages tdes_batch_submit_noalloc takes.
BATCH_NOALLOC_MAX_MSGS = 1 << 20


def batch_submit_noalloc_ptr(d_msgs, n_msgs, d_sched, n_sched, d_in, in_bytes, d_out, out_bytes,
                             d_skipped=0, stream=0):
    """tdes_batch_submit_noalloc on raw device addresses (no workspace;
    d_skipped: device address of a uint64 for the skipped count, or 0)."""
    _check(lib().tdes_batch_submit_noalloc(ctypes.c_void_p(d_msgs), n_msgs,
                                           ctypes.c_void_p(d_sched), n_sched,
                                           ctypes.c_void_p(d_in), in_bytes,
                                           ctypes.c_void_p(d_out), out_bytes,
                                           ctypes.c_void_p(d_skipped or None),
                                           ctypes.c_void_p(stream)))


def batch_get_config():
    """The batched kernel's configuration on the current device (a dict)."""
    c = BatchConfig()
    _check(lib().tdes_batch_get_config(ctypes.byref(c)))
    return c.as_dict()


def batch_set_config(kmax, waves, grid_mult):
    _check(lib().tdes_batch_set_config(ctypes.byref(BatchConfig(kmax, waves, grid_mult, 0))))


def batch_config_load(path, device, cus):
    """The tuning cache's entry for (device, cus) as a dict, or None."""
    c = BatchConfig()
    r = lib().tdes_batch_config_load(path.encode(), device.encode(), cus, ctypes.byref(c))
    if r < 0:
        _check(r)
    return c.as_dict() if r == 1 else None


def batch_config_save(path, device, cus, kmax, waves, grid_mult, us_per_batch=0.0):
    _check(lib().tdes_batch_config_save(path.encode(), device.encode(), cus,
                                        ctypes.byref(BatchConfig(kmax, waves, grid_mult, 0)),
                                        float(us_per_batch)))


def msg_table(in_off, out_off, nbytes, sched_idx, dirs):
    """Descriptor array (numpy, n x 4 int64 = n tdes_msg) from per-message fields."""
    import numpy as np
    n = len(nbytes)
    t = np.zeros((n, 4), dtype=np.uint64)
    t[:, 0] = np.asarray(in_off, dtype=np.uint64)
    t[:, 1] = np.asarray(out_off, dtype=np.uint64)
    t[:, 2] = np.asarray(nbytes, dtype=np.uint64)
    t[:, 3] = (np.asarray(sched_idx, dtype=np.uint64) |
               (np.asarray(dirs, dtype=np.uint64) << np.uint64(32)))
    return t.view(np.int64)


class Batch:
    """Device-resident pieces of one batch: descriptors, key schedules and
    workspace (torch tensors), built once and submitted any number of times."""

    def __init__(self, keys, in_off, out_off, nbytes, dirs, sched_idx=None, stream=None):
        import numpy as np
        import torch
        n = len(nbytes)
        if sched_idx is None:
            sched_idx = np.arange(n)
        sch = key_schedules(keys)
        self.n_msgs, self.n_sched = n, len(sch)
        self.sched = torch.empty(len(sch) * DEVICE_SCHEDULE_BYTES, dtype=torch.uint8, device="cuda")
        self.stream = _stream_handle(stream)
        schedule_upload(sch, self.sched.data_ptr(), self.stream)
        table = msg_table(in_off, out_off, nbytes, sched_idx, dirs)
        self.msgs = torch.from_numpy(table).to("cuda")
        self.ws_bytes = batch_workspace_bytes(n)
        self.ws = torch.empty((self.ws_bytes + 7) // 8, dtype=torch.int64, device="cuda")

    def submit(self, x, out, stream=None):
        """Run the batch over input base x and output base out (uint8 CUDA
        tensors; message ranges are checked against their sizes)."""
        batch_submit_ptr(self.msgs.data_ptr(), self.n_msgs, self.sched.data_ptr(), self.n_sched,
                         x.data_ptr(), x.numel(), out.data_ptr(), out.numel(),
                         self.ws.data_ptr(), self.ws_bytes,
                         _stream_handle(stream) if stream is not None else self.stream)
        return out

    def autotune(self, x, out, reps=3, stream=None):
        """Time this batch in every batched-kernel configuration and keep the
        fastest for later batched launches on this device (and in the tuning
        cache); returns it as a dict (synchronous).  x and out must not
        overlap."""
        c = BatchConfig()
        _check(lib().tdes_batch_autotune(
            ctypes.c_void_p(self.msgs.data_ptr()), self.n_msgs, ctypes.c_void_p(self.sched.data_ptr()),
            self.n_sched, ctypes.c_void_p(x.data_ptr()), x.numel(),
            ctypes.c_void_p(out.data_ptr()), out.numel(),
            ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
            ctypes.c_void_p(_stream_handle(stream) if stream is not None else self.stream),
            int(reps), ctypes.byref(c)))
        return c.as_dict()

    def autotune_streams(self, x, outs, streams, reps=3):
        """The autotuner for a stream of these batches over several streams
        (tdes_batch_autotune_streams): lane i writes outs[i] on streams[i]
        (torch streams) with a workspace of its own; returns the kept
        configuration as a dict (synchronous).  The outputs must not overlap
        x or each other."""
        import torch
        n = len(outs)
        if n != len(streams) or n < 1:
            raise ValueError("one output per stream")
        wss = [self.ws] + [torch.empty_like(self.ws) for _ in range(n - 1)]
        arr = lambda v: (ctypes.c_void_p * n)(*[ctypes.c_void_p(p) for p in v])
        c = BatchConfig()
        size = outs[0].numel()
        if any(o.numel() != size for o in outs):
            raise ValueError("outputs of one size")
        _check(lib().tdes_batch_autotune_streams(
            ctypes.c_void_p(self.msgs.data_ptr()), self.n_msgs,
            ctypes.c_void_p(self.sched.data_ptr()), self.n_sched, ctypes.c_void_p(x.data_ptr()),
            x.numel(), arr([o.data_ptr() for o in outs]), size,
            arr([w.data_ptr() for w in wss]), self.ws_bytes,
            arr([_stream_handle(st) for st in streams]), n, int(reps), ctypes.byref(c)))
        return c.as_dict()

    def skipped(self):
        """Messages the last submit skipped as invalid (synchronises)."""
        return int(self.ws[1].item())
