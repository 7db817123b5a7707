"""Algorithmic work per 64-bit block of each kernel, for roofline figures.

Counted from the generated code, in 32-bit VALU lane operations (one
v_bitop3_b32 / v_xor_b32 / v_perm_b32 ... on one lane):

bitsliced (per 32 blocks = one lane):
  48 rounds x (S-box gates + 32 three-input XORs of the outputs into the other
  half, which also carry the key masks, + key XORs of the second-use inputs
  whose masks are not folded into their gates: BS_XORS_PER_ROUND in all)
  + 4 transposes of 32 words (2 in, 2 out), each 16 pairs x
    (2 + 2 + 4 + 4 + 4) ops (byte stages: one v_perm_b32 per word; bit
    stages: two shifts, or a shift and an addition, and two v_bitop3_b32
    selects per pair)
  IP, E, P and FP are register renaming: no operations.
table (SP-box) kernel (per block):
  48 rounds x (1 rotate + 4 key XORs + 6 shifts and 8 mask-and-offset ops
  that turn the 8 windows into LDS addresses + 4 three-input XORs folding
  the 8 table words into the other half)
  + IP and FP as delta swaps (the operation counts the generator writes
  beside them); plus 8 LDS reads a round.
HBM traffic: every block is read once and written once: 16 bytes.
"""
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
GEN = os.path.join(HERE, "csrc", "generated")

# MI355X: 256 CUs x 4 SIMDs x 32 lanes/clock x 2.4 GHz, 32-bit VALU lane-ops/s.
# Wave64 bitwise VALU instructions issue at 32 lanes per clock per SIMD (two
# waves' instructions per 4-clock window); the probe kernels in
# include/tdes_probe.h sustain 55-60 T under load (v_xor_b32, v_bitop3_b32,
# at a lower shader clock), above the 39.3 T that 16 lanes per clock would
# allow at 2.4 GHz.
VALU_PEAK_OPS = 256 * 4 * 32 * 2.4e9
HBM_PEAK_BYTES = 8.0e12
HBM_BYTES_PER_BLOCK = 16
TRANSPOSE_OPS = 16 * (2 + 2 + 4 + 4 + 4)


def _read(name):
    with open(os.path.join(GEN, name)) as f:
        return f.read()


def sbox_gates_per_round():
    m = re.search(r"#define BS_SBOX_GATES_PER_ROUND (\d+)", _read("bitslice_gen.h"))
    return int(m.group(1))


def xors_per_round():
    m = re.search(r"#define BS_XORS_PER_ROUND (\d+)", _read("bitslice_gen.h"))
    return int(m.group(1))


def bitslice_ops_per_block():
    per_lane = 48 * (sbox_gates_per_round() + xors_per_round()) + 4 * TRANSPOSE_OPS
    return per_lane / 32.0


def spbox_ops_per_block():
    text = _read("spbox_gen.h")
    ipfp = sum(int(g) for g in re.findall(r"\((\d+) operations\)", text))
    return 48 * (1 + 4 + 6 + 8 + 4) + ipfp


def ops_per_block(kernel):
    return spbox_ops_per_block() if kernel == "spbox" else bitslice_ops_per_block()
