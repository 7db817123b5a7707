"""S-box gate networks: text format, evaluation and exhaustive verification.

A network computes one DES S-box (Sec. III-B, S-box step) with 3-input
lookup-table gates.  Signals 0..5 are the six S-box inputs b1..b6; gate i
(numbered from 6) is ``LUT3(a, b, c, imm)``, whose value is bit
``(a << 2) | (b << 1) | c`` of ``imm`` (the v_bitop3_b32 convention).  The
four outputs are signals, optionally complemented, giving the S-box value
most significant bit first.
"""
import os

from .des_tables import SBOX

HERE = os.path.dirname(os.path.abspath(__file__))
NETWORKS_PATH = os.path.join(HERE, "sbox_networks.txt")


def lut3(imm, a, b, c):
    """Evaluate the gate on plain 0/1 values."""
    return (imm >> ((a << 2) | (b << 1) | c)) & 1


def parse_network(text):
    gates, outs = [], [None] * 4
    for line in text.splitlines():
        f = line.split()
        if not f:
            continue
        if f[0] == "g":
            idx, a, b, c, imm = (int(x) for x in f[1:6])
            assert idx == 6 + len(gates), "gates must be numbered in order"
            assert max(a, b, c) < idx, "gate reads a later signal"
            gates.append((a, b, c, imm))
        elif f[0] == "out":
            q, sig, neg = (int(x) for x in f[1:4])
            outs[q] = (sig, neg)
    assert all(o is not None for o in outs)
    return {"gates": gates, "outs": outs}


def evaluate(net, v):
    """Outputs (4-bit value, MSB first) of the network on 6-bit input v
    (b1 is bit 5 of v)."""
    sig = [(v >> (5 - q)) & 1 for q in range(6)]
    for a, b, c, imm in net["gates"]:
        sig.append(lut3(imm, sig[a], sig[b], sig[c]))
    val = 0
    for sgn, neg in net["outs"]:
        val = (val << 1) | (sig[sgn] ^ neg)
    return val


def sbox_value(box, v):
    """S-box ``box`` (0..7) on the 6-bit chunk v: row from the outer bits,
    column from the middle four (Sec. III-B)."""
    row = ((v >> 5) << 1) | (v & 1)
    col = (v >> 1) & 0xF
    return SBOX[box][row][col]


def verify_network(box, net):
    """Exhaustive check over all 64 inputs; raises on any mismatch."""
    for v in range(64):
        got, want = evaluate(net, v), sbox_value(box, v)
        if got != want:
            raise AssertionError("S%d network wrong at input %d: %d != %d" % (box + 1, v, got, want))


def format_networks(nets):
    lines = ["# DES S-box gate networks (3-input LUT gates, v_bitop3_b32 tables).",
             "# Written by synth_sboxes.py; checked exhaustively by networks.verify_network.",
             "# box <n> <gates>; g <signal> <a> <b> <c> <imm>; out <bit> <signal> <complemented>"]
    for box in sorted(nets):
        net = nets[box]
        lines.append("box %d %d" % (box, len(net["gates"])))
        for i, (a, b, c, imm) in enumerate(net["gates"]):
            lines.append("g %d %d %d %d %d" % (6 + i, a, b, c, imm))
        for q, (sig, neg) in enumerate(net["outs"]):
            lines.append("out %d %d %d" % (q, sig, neg))
    return "\n".join(lines) + "\n"


def load_networks(path=NETWORKS_PATH):
    nets, cur, box = {}, [], None
    with open(path) as f:
        for line in f:
            s = line.split("#")[0].strip()
            if not s:
                continue
            if s.startswith("box "):
                if box is not None:
                    nets[box] = parse_network("\n".join(cur))
                box, cur = int(s.split()[1]), []
            else:
                cur.append(s)
    if box is not None:
        nets[box] = parse_network("\n".join(cur))
    return nets
