"""Build libtdes.so in-tree with hipcc for gfx950.

    python -m paper_2007_10752_amd.build [-v]

Regenerates csrc/generated from the tables and the committed S-box networks
(deterministic, fast), compiles every source to an object and links the
shared library next to this file.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libtdes.so")
SOURCES = ("api.cpp", "keysched.cpp", "serve.cpp", "host_path.cpp", "batch_tune.cpp",
           "bitslice.hip", "batch.hip",
           "spbox.hip", "probe.hip", "replica.hip")
ARCH = os.environ.get("TDES_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH,
          # no packed-FP32 instructions anywhere in device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False, sanitize=None):
    """Build the library.  sanitize (e.g. "address,undefined" or "thread")
    instruments the host code only, for CPU test runs, and writes
    _build/<name>/libtdes.so instead of the package's library; device code
    is compiled as usual."""
    from .gen import emit
    emit.main() if verbose else _quiet(emit.main)
    out_dir = BUILD_DIR if not sanitize else \
        os.path.join(BUILD_DIR, "san_" + sanitize.replace(",", "_"))
    lib = LIB if not sanitize else os.path.join(out_dir, "libtdes.so")
    os.makedirs(out_dir, exist_ok=True)
    # -Xarch_host: the sanitizer applies to host code, never to GPU code
    san = ["-Xarch_host", "-fsanitize=" + sanitize, "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xarch_host", "-g"] if sanitize else []
    objs = []
    for src in SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        cmd = [HIPCC] + COMMON + san + (DEVICE if src.endswith(".hip") else []) + \
              ["-c", os.path.join(CSRC, src), "-o", obj]
        _run(cmd, verbose)
        objs.append(obj)
    tmp = lib + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + san + objs, verbose)
    os.replace(tmp, lib)
    return lib


def _quiet(fn):
    import contextlib
    import io
    with contextlib.redirect_stdout(io.StringIO()):
        fn()


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
