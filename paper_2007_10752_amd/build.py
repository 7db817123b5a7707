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
SOURCES = ("api.cpp", "keysched.cpp", "serve.cpp", "host_path.cpp", "bitslice.hip", "batch.hip",
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


def build(verbose=False):
    from .gen import emit
    emit.main() if verbose else _quiet(emit.main)
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        cmd = [HIPCC] + COMMON + (DEVICE if src.endswith(".hip") else []) + \
              ["-c", os.path.join(CSRC, src), "-o", obj]
        _run(cmd, verbose)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


def _quiet(fn):
    import contextlib
    import io
    with contextlib.redirect_stdout(io.StringIO()):
        fn()


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
