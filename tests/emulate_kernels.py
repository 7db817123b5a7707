"""CPU emulation of the two HIP kernels' arithmetic, built from the same
generated headers the kernels compile (renaming maps, gate networks, SP
tables, IP/FP code) and the same key formats.  Used by the host tests to
check the generator and the key formats before anything runs on a GPU; the
GPU parity tests then check the hardware path itself.
"""
import os
import re

import numpy as np

from paper_2007_10752_amd.gen import emit
from paper_2007_10752_amd.gen.networks import load_networks

GEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2007_10752_amd", "csrc", "generated")
M32 = 0xFFFFFFFF


def _header(name):
    with open(os.path.join(GEN, name)) as f:
        return f.read()


def _int_array(text, name):
    m = re.search(r"%s\[\d+\] = \{([^}]*)\}" % name, text)
    return [int(v, 0) for v in m.group(1).replace("u", "").split(",") if v.strip()]


# ------------------------------------------------------------ bitsliced ----

def _lut3(imm, a, b, c):
    r = 0
    for idx in range(8):
        if (imm >> idx) & 1:
            r |= (a if idx & 4 else ~a) & (b if idx & 2 else ~b) & (c if idx & 1 else ~c)
    return r & M32


def _transpose32(x):
    return [sum(((x[b] >> p) & 1) << b for b in range(32)) for p in range(32)]


def _bs_masks(key_bytes, box_dup, c):
    """Expand the kernel's 100 key-mask words into its LDS layout: round t,
    box j, slot s at kBsRoundMasks*t + kBsBoxMasks*j + s is bit 4j + s of
    word 2t (s < 4) or bit box_dup[4j + s - 4] of word 2t + 1 (s >= 4, 0 if
    that is -1); extra group g, entry n at kBsInitY + 32g + n is bit n of
    word 96 + g."""
    w = [int(v) for v in np.frombuffer(key_bytes, dtype="<u4")]
    assert len(w) == 100
    bit = lambda word, b: M32 if (w[word] >> b) & 1 else 0
    out = [0] * c["kBsNumMasks"]
    for t in range(48):
        for j in range(8):
            base = c["kBsRoundMasks"] * t + c["kBsBoxMasks"] * j
            for q in range(4):
                out[base + q] = bit(2 * t, 4 * j + q)
            for i in range(4):
                k = box_dup[4 * j + i]
                out[base + 4 + i] = 0 if k < 0 else bit(2 * t + 1, k)
    for g in range(4):
        for n in range(32):
            out[c["kBsInitY"] + 32 * g + n] = bit(96 + g, n)
    return out


def _int_const(text, name):
    return int(re.search(r"%s = (\d+)" % name, text).group(1))


_OPERAND = re.compile(r"^(?:r\[(\d+)\]|d\[(\d+)\]|m\.o\[(\d+)\]|m\.e\[(\d+)\]|(\w+))$")


def _operand(text):
    m = _OPERAND.match(text.strip())
    assert m, text
    for kind, g in zip(("r", "d", "o", "e"), m.groups()[:4]):
        if g is not None:
            return (kind, int(g))
    return ("v", m.group(5))


def _piped_round_boxes(text):
    """The statements of the generated bs_round_piped, per S-box: (box,
    [(kind, lhs, operands, imm)]) with kind "lut" (v_bitop3_b32) or "xor";
    the mask loads and scheduling barriers are left out."""
    body = text[text.index("void bs_round_piped("):]
    body = body[:body.index("\n}\n")]
    boxes = []
    for line in body.splitlines():
        line = line.strip()
        mb = re.match(r"const BsBoxMasks &m = pm\[(\d+)\];", line)
        if mb:
            boxes.append((int(mb.group(1)), []))
            continue
        ma = re.match(r"(?:const uint32_t )?(\w+|d\[\d+\]) = (.*);(?:\s*//.*)?$", line)
        if not ma or not boxes:
            continue
        lhs, rhs = _operand(ma.group(1)), ma.group(2)
        lhs = ("d", lhs[1]) if lhs[0] == "d" else ("v", lhs[1])
        ml = re.match(r"__builtin_amdgcn_bitop3_b32\((.*), (0x[0-9a-f]+)\)$", rhs)
        if ml:
            ops = [_operand(o) for o in ml.group(1).split(",")]
            boxes[-1][1].append(("lut", lhs, ops, int(ml.group(2), 16)))
        else:
            ops = [_operand(o) for o in rhs.split("^")]
            boxes[-1][1].append(("xor", lhs, ops, 0))
    assert [b for b, _ in boxes] == list(range(8)), [b for b, _ in boxes]
    return boxes


def bitslice_ecb(key_bytes, data):
    """Emulate tdes_bitslice_kernel on up to 32 blocks (one lane), given the
    kernel's key argument (tdes_kernel_key_bytes)."""
    text = _header("bitslice_gen.h")
    ktext = _header("bitslice_keys_gen.h")
    ip_l, ip_r = _int_array(text, "BS_IP_L"), _int_array(text, "BS_IP_R")
    fp_src = _int_array(text, "BS_FP_SRC")
    c = {k: _int_const(ktext, k) for k in ("kBsBoxMasks", "kBsRoundMasks", "kBsInitY",
                                           "kBsRemask16", "kBsRemask32", "kBsFinalX",
                                           "kBsNumMasks")}
    box_dup = _int_array(ktext, "kBsBoxDup")
    km = _bs_masks(key_bytes, box_dup, c)

    d = np.asarray(data, dtype=np.uint8)
    nblk = d.size // 8
    assert nblk <= 32
    words = np.zeros(64, dtype=np.uint32)
    words[:2 * nblk] = d.view("<u4")
    h0 = _transpose32([int(words[2 * b]) for b in range(32)])
    h1 = _transpose32([int(words[2 * b + 1]) for b in range(32)])
    plane = h0 + h1
    X = [plane[i] for i in ip_l]
    Y = [plane[i] ^ km[c["kBsInitY"] + n] for n, i in enumerate(ip_r)]

    boxes = _piped_round_boxes(text)

    def rnd(dst, src, t):
        # the emitted bs_round_piped, statement by statement: box j reads its
        # masks o[q] (slot q) and e[i] (slot 4 + i) of round t
        for box, stmts in boxes:
            m = km[c["kBsRoundMasks"] * t + c["kBsBoxMasks"] * box:]
            env = {}

            def val(tok):
                kind, a = tok
                if kind == "r":
                    return src[a]
                if kind == "d":
                    return dst[a]
                if kind == "o":
                    return m[a]
                if kind == "e":
                    return m[4 + a]
                return env[a]

            for kind, lhs, ops, imm in stmts:
                v = [val(o) for o in ops]
                res = _lut3(imm, *v) if kind == "lut" else (v[0] ^ v[1] if len(v) == 2 else v[0])
                if lhs[0] == "d":
                    dst[lhs[1]] = res
                else:
                    env[lhs[1]] = res

    for t in range(0, 16, 2):
        rnd(X, Y, t)
        rnd(Y, X, t + 1)
    X = [v ^ km[c["kBsRemask16"] + i] for i, v in enumerate(X)]
    for t in range(16, 32, 2):
        rnd(Y, X, t)
        rnd(X, Y, t + 1)
    Y = [v ^ km[c["kBsRemask32"] + i] for i, v in enumerate(Y)]
    for t in range(32, 48, 2):
        rnd(X, Y, t)
        rnd(Y, X, t + 1)
    X = [v ^ km[c["kBsFinalX"] + i] for i, v in enumerate(X)]
    pre = Y + X
    out_planes = [pre[fp_src[q]] for q in range(64)]
    o0, o1 = _transpose32(out_planes[:32]), _transpose32(out_planes[32:])
    ow = np.zeros(64, dtype=np.uint32)
    for b in range(32):
        ow[2 * b], ow[2 * b + 1] = o0[b], o1[b]
    return ow.view(np.uint8)[:8 * nblk].copy()


# ------------------------------------------------------------ table kernel --

def spbox_keys_from_bytes(key_bytes):
    """Per round: odd chunks, even chunks, chunks 0 and 6 and chunk 7 of the
    half rotated left by 12."""
    w = np.frombuffer(key_bytes, dtype="<u4").reshape(48, 4)
    return [list(map(int, w[:, i])) for i in range(4)]


def _rotl(x, s):
    return ((x << s) | (x >> (32 - s))) & M32


def _run_macro(text, name, env):
    """Execute one of the generated IP/FP macros on Python ints (32-bit
    unsigned arithmetic: every variable is reduced mod 2^32 after each
    statement, as C's uint32_t would be)."""
    m = re.search(r"#define %s\([^)]*\) do \{ \\\n(.*?)\} while \(0\)" % name, text, re.S)
    glb = {"rotr": lambda x, s: ((x >> s) | (x << (32 - s))) & M32,
           "bswap": lambda x: int.from_bytes(int(x).to_bytes(4, "little"), "big")}
    for line in m.group(1).split("\\\n"):
        for stmt in line.split(";"):
            stmt = stmt.strip()
            if not stmt:
                continue
            stmt = re.sub(r"__builtin_amdgcn_alignbit\((\w+), \w+, (\d+)\)",
                          lambda mm: "rotr(%s, %s)" % (mm.group(1), mm.group(2)), stmt)
            stmt = stmt.replace("__builtin_bswap32", "bswap")
            stmt = re.sub(r"(0x[0-9a-f]+)u", r"\1", stmt)
            stmt = re.sub(r"\b(\d+)u\b", r"\1", stmt)
            if stmt.startswith("uint32_t "):
                # a declaration: "uint32_t a = X, b = Y, t"
                decls = []
                for part in stmt[len("uint32_t "):].split(", "):
                    if "=" in part:
                        decls.append(part)
                for d in decls:
                    exec(d, glb, env)
            else:
                exec(stmt, glb, env)
            for k, v in list(env.items()):
                if isinstance(v, int):
                    env[k] = v & M32
    return env


def spbox_ecb(key_bytes, data):
    """Emulate tdes_spbox_kernel block by block, given its key argument."""
    text = _header("spbox_gen.h")
    sp = _int_array(text, "SP_TABLE")
    ko, ke, k06, k7 = spbox_keys_from_bytes(key_bytes)

    def f(R, r):
        ro, re_, rr = R ^ ko[r], R ^ ke[r], _rotl(R, 12)
        a06, a7 = rr ^ k06[r], rr ^ k7[r]
        idx = [(a06 >> 7) & 63, (ro >> 23) & 63, (re_ >> 19) & 63, (ro >> 15) & 63,
               (re_ >> 11) & 63, (ro >> 7) & 63, (a06 >> 15) & 63, (a7 >> 11) & 63]
        v = 0
        for s in range(8):
            v ^= sp[64 * s + idx[s]]
        return v

    d = np.asarray(data, dtype=np.uint8)
    w = d.view("<u4")
    out = np.zeros_like(w)
    for b in range(d.size // 8):
        env = _run_macro(text, "SP_IP", {"w0": int(w[2 * b]), "w1": int(w[2 * b + 1])})
        X, Y = env["L"], env["R"]
        for r in range(0, 16, 2):
            X ^= f(Y, r)
            Y ^= f(X, r + 1)
        for r in range(16, 32, 2):
            Y ^= f(X, r)
            X ^= f(Y, r + 1)
        for r in range(32, 48, 2):
            X ^= f(Y, r)
            Y ^= f(X, r + 1)
        env = _run_macro(text, "SP_FP", {"Lf": X, "Rf": Y})
        out[2 * b], out[2 * b + 1] = env["o0"], env["o1"]
    return out.view(np.uint8).copy()


def generated_headers_match():
    """True if the committed headers equal what the emitter writes now."""
    nets = load_networks()
    want = {"des_tables_gen.h": emit.emit_tables(), "bitslice_gen.h": emit.emit_bitslice(nets),
            "bitslice_keys_gen.h": emit.emit_bitslice_keys(), "spbox_gen.h": emit.emit_spbox(),
            "replica_tables_gen.h": emit.emit_replica_tables()}
    return {name: _header(name) == text for name, text in want.items()}
