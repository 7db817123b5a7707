"""Triple-DES (EDE) over independent 64-bit blocks on AMD Instinct MI355X.

The cipher runs in hand-written HIP kernels behind the C ABI of libtdes.so
(include/tdes.h); ``tdes`` is its ctypes binding, ``workloads`` the seeded
synthetic inputs, ``build`` the in-tree build.
"""
from . import tdes  # noqa: F401  (loads the library lazily, on first call)
