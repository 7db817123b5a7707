"""Transcription checks of the oracle's copy of the Appendix A arrays.

Each check is a structural fact of DES that a mistyped entry would break:
the permutations are bijections, the initial permutation has the printed
column/row (bit-matrix transpose) structure and the final permutation is its
inverse, the expansion takes overlapping 6-bit windows of the right half,
the rotations add up to one full turn of each 28-bit half, and so on.
"""
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def t(name):
    return oracle.table(name)


def test_lengths():
    sizes = {"pc_1": 56, "shift_keys": 16, "pc_2": 48, "initial_perm": 64,
             "exp_d": 48, "s": 512, "per": 32, "final_perm": 64}
    for name, n in sizes.items():
        assert len(t(name)) == n, name


def test_pc1_drops_exactly_the_parity_bits():
    # Sec. III-A: the 64-bit key is reduced to 56 bits; the 8 bits not taken
    # are the parity bits 8, 16, ..., 64.
    pc1 = t("pc_1")
    assert len(set(pc1)) == 56
    assert set(range(1, 65)) - set(pc1) == {8 * i for i in range(1, 9)}


def test_shifts_add_to_one_turn():
    # 16 rotations of a 28-bit half that return it to its start (so round
    # key 16 is PC-2 of the unrotated halves).
    sk = t("shift_keys")
    assert sum(sk) == 28 and set(sk) <= {1, 2}


def test_pc2_takes_24_bits_from_each_half():
    pc2 = t("pc_2")
    assert len(set(pc2)) == 48 and min(pc2) >= 1 and max(pc2) <= 56
    assert all(v <= 28 for v in pc2[:24])
    assert all(v > 28 for v in pc2[24:])


def test_initial_perm_is_a_bit_matrix_transpose():
    # Output row r (8 bits) gathers one input bit column, from byte 8 down
    # to byte 1: even columns 2, 4, 6, 8 first, then odd columns 1, 3, 5, 7.
    ip = t("initial_perm")
    cols = [2, 4, 6, 8, 1, 3, 5, 7]
    for r in range(8):
        for c in range(8):
            assert ip[8 * r + c] == 8 * (7 - c) + cols[r]


def test_final_perm_inverts_initial_perm():
    ip, fp = t("initial_perm"), t("final_perm")
    assert sorted(fp) == list(range(1, 65))
    for j in range(64):
        assert ip[fp[j] - 1] == j + 1
        assert fp[ip[j] - 1] == j + 1


def test_expansion_is_overlapping_windows():
    # Chunk s (0..7) takes right-half bits 4s .. 4s+5 (1-based, cyclic), so
    # neighbouring chunks share two bits.
    e = t("exp_d")
    for s in range(8):
        for q in range(6):
            assert e[6 * s + q] == (4 * s + q - 1) % 32 + 1


def test_straight_permutation_is_a_bijection():
    assert sorted(t("per")) == list(range(1, 33))


def test_sbox_rows_are_permutations():
    s = t("s")
    for box in range(8):
        for row in range(4):
            cells = s[64 * box + 16 * row: 64 * box + 16 * row + 16]
            assert sorted(cells) == list(range(16)), (box, row)


def test_sbox_single_bit_input_change_moves_two_output_bits():
    # A published design property of the DES S-boxes: inputs that differ in
    # exactly one bit give outputs that differ in at least two bits.
    for box in range(8):
        vals = [oracle.sbox(box, v) for v in range(64)]
        for v in range(64):
            for b in range(6):
                assert bin(vals[v] ^ vals[v ^ (1 << b)]).count("1") >= 2
