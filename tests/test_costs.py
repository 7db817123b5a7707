"""The roofline's operation count is the generated code's: the piped round
holds one v_bitop3_b32 per S-box gate plus 32 output XORs (which also carry
the key masks), and one plain XOR per second-use input whose mask is not
folded into its gates (16 second uses a round); with four 256-operation
transposes per 32 blocks that is (48 x (gates + XORs) + 1024) / 32 lane
operations per block."""
import os
import re

from paper_2007_10752_amd import costs

GEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2007_10752_amd", "csrc", "generated", "bitslice_gen.h")


def _piped_round_body():
    text = open(GEN).read()
    start = text.index("bs_round_piped(")
    end = text.index("\n}\n", start)
    return text[start:end]


def test_ops_per_round_match_generated_code():
    body = _piped_round_body()
    gates = costs.sbox_gates_per_round()
    xors = len(re.findall(r"\^ m\.e\[", body))
    folded = len(re.findall(r"mask folded into its gates", body))
    assert body.count("__builtin_amdgcn_bitop3_b32(") == gates + 32
    assert xors + folded == 16
    assert costs.xors_per_round() == 32 + xors
    # a folded mask is read by gates only, as their third operand
    assert len(re.findall(r"bitop3_b32\([^;]*m\.e\[", body)) >= folded


def test_ops_per_block():
    gates = costs.sbox_gates_per_round()
    xors = costs.xors_per_round()
    assert costs.TRANSPOSE_OPS == 256
    want = (48 * (gates + xors) + 4 * 256) / 32
    assert abs(costs.ops_per_block("bitslice") - want) < 1e-9
    if gates == 196 and xors == 46:
        assert costs.ops_per_block("bitslice") == 395
