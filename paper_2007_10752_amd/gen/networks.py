"""S-box gate networks: text format, evaluation and exhaustive verification.

A network computes one DES S-box (Sec. III-B, S-box step) with 3-input
lookup-table gates.  Signals 0..5 are the six S-box inputs b1..b6; gate i
(numbered from 6) is ``LUT3(a, b, c, imm)``, whose value is bit
``(a << 2) | (b << 1) | c`` of ``imm`` (the v_bitop3_b32 convention).  The
four outputs are signals, optionally complemented, giving the S-box value
most significant bit first.
"""
import itertools
import os

from .des_tables import E, SBOX

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


# ------------------------------------------------ key masks in the gates --
#
# In the bitsliced kernel an S-box input is a right-half word XORed with a
# key mask (0 or all ones).  Each half word carries the mask of one of its
# expansion positions already (its primary use); the 16 words the expansion
# reads twice need an XOR with a second mask at their other position (the
# second use).  That XOR can be folded into the network when every gate that
# depends on the input depends on one other signal at most: the gate then
# takes the raw word, the other signal and the mask, and computes its
# function of (word ^ mask).  Which of a word's two positions is the second
# use is free; second_use_plan picks it so that as many second uses as
# possible fold.

MASK_BASE = 100  # signal MASK_BASE + q: the key mask of input q in a folded network


def live_signals(gate):
    """The signals a gate's value depends on (a signal in two slots counts
    once, with both slots taking its value)."""
    a, b, c, imm = gate
    sig = sorted({a, b, c})
    live = set()
    for sg in sig:
        for bits in itertools.product((0, 1), repeat=len(sig)):
            val = dict(zip(sig, bits))
            v0 = lut3(imm, val[a], val[b], val[c])
            val[sg] ^= 1
            if lut3(imm, val[a], val[b], val[c]) != v0:
                live.add(sg)
                break
    return live


def foldable(net, inputs):
    """Can the masks of all `inputs` (S-box input indices) enter the network
    through the gates that read them?"""
    inputs = set(inputs)
    if any(sig in inputs for sig, _ in net["outs"]):
        return False
    for g in net["gates"]:
        live = live_signals(g)
        mine = live & inputs
        if mine and (len(live) > 2 or len(mine) > 1):
            return False
    return True


def fold_network(net, inputs):
    """The network with the masks of `inputs` taken by their gates: signal
    q of a folded input is the raw word, MASK_BASE + q its mask; a gate that
    depends on it becomes LUT3(q, other, MASK_BASE + q).  Gates that do not
    depend on a folded input keep their operands (a dead operand q is then
    the raw word, which the gate ignores)."""
    assert foldable(net, inputs)
    inputs = set(inputs)
    gates = []
    for g in net["gates"]:
        a, b, c, imm = g
        live = live_signals(g)
        mine = live & inputs
        if not mine:
            gates.append(g)
            continue
        q = mine.pop()
        rest = sorted(live - {q})
        y = rest[0] if rest else q
        new_imm = 0
        for idx in range(8):
            r, yv, m = (idx >> 2) & 1, (idx >> 1) & 1, idx & 1
            val = {q: r ^ m}
            if y != q:
                val[y] = yv
            ops = [val.get(x, 0) for x in (a, b, c)]
            new_imm |= lut3(imm, *ops) << idx
        gates.append((q, y, MASK_BASE + q, new_imm))
    return {"gates": gates, "outs": list(net["outs"]), "folded": sorted(inputs)}


def verify_folded(box, fnet):
    """Exhaustive check of a folded network: for every value of the words the
    kernel holds and every value of the folded inputs' masks, the outputs are
    the S-box of the masked input."""
    folded = fnet["folded"]
    for v in range(64):
        for mbits in range(1 << len(folded)):
            sig = {q: (v >> (5 - q)) & 1 for q in range(6)}
            eff = v
            for i, q in enumerate(folded):
                m = (mbits >> i) & 1
                sig[MASK_BASE + q] = m
                eff ^= m << (5 - q)
            for i, (a, b, c, imm) in enumerate(fnet["gates"]):
                sig[6 + i] = lut3(imm, sig[a], sig[b], sig[c])
            got = 0
            for sg, neg in fnet["outs"]:
                got = (got << 1) | (sig[sg] ^ neg)
            if got != sbox_value(box, eff):
                raise AssertionError("S%d folded network wrong at input %d, masks %d"
                                     % (box + 1, v, mbits))


def shared_words():
    """The 16 right-half words the expansion reads twice: for each, its two
    positions e (0..47, S-box e // 6, input e % 6) in e order."""
    pos = {}
    for e in range(48):
        pos.setdefault(E[e] - 1, []).append(e)
    return [tuple(p) for j, p in sorted(pos.items()) if len(p) == 2]


def second_use_plan(nets):
    """Choose, for each word read twice, which position is its second use,
    and which second uses fold into their S-box's gates.  Maximises the
    folded count; among equal plans keeps the most second uses at the later
    position in e order.  Returns (second-use positions, folded positions),
    both sets of e."""
    shared = shared_words()
    cand = {}  # box -> shared inputs of that box
    for pair in shared:
        for e in pair:
            cand.setdefault(e // 6, []).append(e % 6)
    options = []
    for box in range(8):
        qs = sorted(cand.get(box, []))
        opts = [frozenset(c) for n in range(len(qs) + 1)
                for c in itertools.combinations(qs, n) if foldable(nets[box], c)]
        options.append(opts)
    # each box has a handful of fold options at most (a fold needs a free
    # operand in every gate that reads the input); keep the search bounded
    # all the same by dropping the smaller options of the widest boxes
    while True:
        size = 1
        for o in options:
            size *= len(o)
        if size <= 1 << 20:
            break
        widest = max(range(8), key=lambda b: len(options[b]))
        options[widest] = sorted(options[widest], key=len)[len(options[widest]) // 2:]
    best, best_key = None, None
    for choice in itertools.product(*options):
        fold_e = {6 * box + q for box, c in enumerate(choice) for q in c}
        covered, second, moved = set(), set(), 0
        ok = True
        for first, later in shared:
            if later in fold_e:
                second.add(later)
                covered.add(later)
            elif first in fold_e:
                second.add(first)
                covered.add(first)
                moved += 1
            else:
                second.add(later)
        # a choice that folds both positions of one word folds one of them for nothing
        if any(a in fold_e and b in fold_e for a, b in shared):
            ok = False
        if not ok:
            continue
        key = (len(covered), -moved)
        if best_key is None or key > best_key:
            best_key, best = key, (second, covered)
    return best


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
