"""The host code of the library under sanitizers, on the CPU.

Two extra builds instrument the host code only (device code is compiled as
usual): AddressSanitizer with UndefinedBehaviorSanitizer, and
ThreadSanitizer.  The host-side test files then run in a child process
against each build (TDES_LIB names it), with the sanitizer's runtime
preloaded into the interpreter: argument checks, key formats, the request
server's scheduler and arena in its host test mode, and concurrent calls
from several threads.  Any report fails the run (halt_on_error)."""
import os
import subprocess
import sys

import pytest

from paper_2007_10752_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"
HOST_TESTS = ["tests/test_host_abi.py", "tests/test_serve_host.py", "tests/test_host_threads.py"]


def _runtime(name):
    if not os.path.exists(CLANG):
        pytest.skip("no clang to locate the sanitizer runtime")
    path = subprocess.run([CLANG, "-print-file-name=libclang_rt.%s-x86_64.so" % name],
                          capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("sanitizer runtime %s not found" % name)
    return path


@pytest.mark.parametrize("sanitize,runtime,marker", [
    ("address,undefined", "asan", "__asan_"),
    ("thread", "tsan", "__tsan_"),
])
def test_host_code_under_sanitizer(sanitize, runtime, marker, tmp_path):
    rt = _runtime(runtime)
    lib = B.build(sanitize=sanitize)
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True,
                          text=True).stdout
    assert marker in syms, "library was not instrumented"
    log = str(tmp_path / "report")
    env = dict(os.environ)
    env.update({
        "TDES_LIB": lib,
        "LD_PRELOAD": rt,
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:log_path=" + log,
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:log_path=" + log,
        "TSAN_OPTIONS": "halt_on_error=1:log_path=" + log,
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu"] + HOST_TESTS, cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    reports = [open(os.path.join(tmp_path, f)).read() for f in sorted(os.listdir(tmp_path))
               if f.startswith("report")]
    assert r.returncode == 0 and not reports, (r.stdout[-3000:], r.stderr[-3000:], reports)
