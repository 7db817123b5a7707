"""Write ecb_1gib_digest.txt: the SHA-256 of the oracle's 3DES-EDE ECB
encryption (Sec. III-B; ECB over every 8-byte block, Sec. V) of the 1 GiB
uniform-random input the benchmark and the GPU parity test use (data seed
SEED_BASE + 2, key seed SEED_BASE + 2 + KEY_SEED_OFFSET).

Calls only the oracle and the seeded input generators:

    python tests/golden/make_ecb_1gib_digest.py

takes about a minute on 8 host threads.  The GPU test compares the digest of
the GPU's full output with the one stored here, so all 134,217,728 blocks are
checked without a full oracle run at test time.
"""
import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2007_10752_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "ecb_1gib_digest.txt")
NBYTES = 1 << 30
CHUNK = 64 << 20


def main():
    t0 = time.time()
    data_seed = W.SEED_BASE + 2
    key_seed = W.SEED_BASE + 2 + W.KEY_SEED_OFFSET
    key = W.key_bundle(W.rng(key_seed))
    data = W.uniform_bytes(W.rng(data_seed), NBYTES)
    h_in = hashlib.sha256(data.tobytes()).hexdigest()
    h_out = hashlib.sha256()
    for off in range(0, NBYTES, CHUNK):
        h_out.update(oracle.tdes_ecb(key, data[off:off + CHUNK]).tobytes())
    with open(OUT, "w") as f:
        f.write("# 3DES-EDE ECB encryption of the 1 GiB uniform input, computed by the oracle\n")
        f.write("# (written by make_ecb_1gib_digest.py; fields: name value)\n")
        f.write("nbytes %d\n" % NBYTES)
        f.write("data_seed %d\n" % data_seed)
        f.write("key_seed %d\n" % key_seed)
        f.write("key24 %s\n" % bytes(key).hex())
        f.write("input_sha256 %s\n" % h_in)
        f.write("encrypt_sha256 %s\n" % h_out.hexdigest())
    print("wrote %s in %.1f s" % (OUT, time.time() - t0))


if __name__ == "__main__":
    main()
