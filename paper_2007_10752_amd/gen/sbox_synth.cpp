// Randomised search for small 3-input-LUT gate networks that compute a DES
// S-box (6 inputs -> 4 outputs), for the bitsliced kernel.
//
// Each signal is a 64-bit truth table over the 6 S-box inputs (bit v of a
// table is the signal's value when the inputs read v, with the first input
// b1 as bit 5 of v).  A gate is an arbitrary boolean function of three
// signals, encoded as the 8-bit table that CDNA4's v_bitop3_b32 takes:
// result bit = imm[(a << 2) | (b << 1) | c].  Complemented operands are free
// (the consumer's table absorbs them), so signals are matched up to
// complement.
//
// Search (written for this project): to realise a target function on a set
// of care positions, reuse an existing signal if one matches, else find one
// gate over any three existing signals, else split the care set on a
// selector signal, realise one side recursively, and join it with a second
// recursively built signal through one more gate whose table is chosen from
// all 16 two-input joins on the other side.  Outputs are built in random
// order with random tie-breaking; the smallest network over many restarts
// wins.  The result is checked exhaustively here and again by the Python
// emitter.
//
// Restricted inputs (SBOX_RESTRICT, a bit mask of inputs 0..5): such an
// input may enter only gates whose other live operand is one signal, so that
// the kernel can pass the key mask the input needs in the free third slot
// (the gate then computes its function of input ^ mask) instead of XORing
// it in first.  Restricted inputs are never reused as signals, selectors or
// operands of three-signal gates; where no other signal splits a care set,
// the search adds a copy gate of a restricted input (the same cost as the
// XOR it would save).
//
// Usage: sbox_synth <restarts> <seed> <box table: 64 values, row-major 4x16>
// Prints the best network as text.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

typedef uint64_t u64;

struct Gate {
    int a, b, c, imm;
};
struct Ref {
    int idx;  // -1: don't care
    int neg;
};

static u64 lut3(int imm, u64 a, u64 b, u64 c) {
    u64 r = 0;
    for (int i = 0; i < 8; i++)
        if ((imm >> i) & 1) r |= ((i & 4) ? a : ~a) & ((i & 2) ? b : ~b) & ((i & 1) ? c : ~c);
    return r;
}

struct Net {
    std::vector<u64> tt;
    std::vector<Gate> g;  // gate i computes tt[6 + i]
    Ref out[4];
};

static std::mt19937_64 rng;
static int g_restrict = 0;
static inline bool restricted(int s) { return s < 6 && ((g_restrict >> s) & 1); }

// Thrown when a restart recurses too deep; the restart is dropped.
struct TooDeep {};

static u64 input_tt(int q) {
    u64 t = 0;
    for (int v = 0; v < 64; v++)
        if ((v >> (5 - q)) & 1) t |= 1ull << v;
    return t;
}

static bool find_existing(const Net &n, u64 t, u64 care, Ref *r) {
    for (int s = (int)n.tt.size() - 1; s >= 0; s--) {
        if (restricted(s)) continue;
        u64 d = (n.tt[s] ^ t) & care;
        if (d == 0) { *r = {s, 0}; return true; }
        if (d == care) { *r = {s, 1}; return true; }
    }
    return false;
}

// One gate over three existing signals that equals t on care.  With
// pick_random, a uniformly random valid triple is returned.
static bool find_single(const Net &n, u64 t, u64 care, Gate *out, bool pick_random) {
    int ns = (int)n.tt.size();
    long found = 0;
    // two-operand gates of a restricted input and one other signal, written
    // LUT3(i, j, j): the kernel puts the mask in the third slot
    for (int i = 0; i < 6; i++) {
        if (!restricted(i)) continue;
        u64 A = n.tt[i];
        for (int j = 0; j < ns; j++) {
            if (j == i || restricted(j)) continue;
            u64 B = n.tt[j];
            int imm = 0, dc = 0;  // 4-entry table, index (a << 1) | b
            bool ok = true;
            for (int p = 0; p < 4 && ok; p++) {
                u64 m = ((p & 2) ? A : ~A) & ((p & 1) ? B : ~B) & care;
                if (!m) { dc |= 1 << p; continue; }
                u64 on = m & t;
                if (on == m) imm |= 1 << p;
                else if (on != 0) ok = false;
            }
            if (!ok) continue;
            found++;
            if (!pick_random || (rng() % found) == 0) {
                imm |= (int)(rng() & 0xf) & dc;
                int imm8 = 0;
                for (int idx = 0; idx < 8; idx++)
                    imm8 |= ((imm >> (idx >> 1)) & 1) << idx;
                *out = {i, j, j, imm8};
                if (!pick_random) return true;
            }
        }
    }
    for (int i = 0; i < ns; i++) {
        if (restricted(i)) continue;
        u64 A = n.tt[i];
        for (int j = i + 1; j < ns; j++) {
            if (restricted(j)) continue;
            u64 B = n.tt[j];
            u64 ab[4] = {~A & ~B & care, ~A & B & care, A & ~B & care, A & B & care};
            // quick reject on the pair alone is not possible in general; go on
            for (int k = j + 1; k < ns; k++) {
                if (restricted(k)) continue;
                u64 C = n.tt[k];
                int imm = 0, dc = 0;
                bool ok = true;
                for (int p = 0; p < 4 && ok; p++) {
                    for (int cb = 0; cb < 2; cb++) {
                        u64 m = ab[p] & (cb ? C : ~C);
                        int idx = (p << 1) | cb;
                        if (!m) { dc |= 1 << idx; continue; }
                        u64 on = m & t;
                        if (on == m) imm |= 1 << idx;
                        else if (on != 0) { ok = false; break; }
                    }
                }
                if (!ok) continue;
                found++;
                if (!pick_random || (rng() % found) == 0) {
                    imm |= (int)(rng() & 0xff) & dc;
                    *out = {i, j, k, imm};
                    if (!pick_random) return true;
                }
            }
        }
    }
    return found > 0;
}

static int add_gate(Net &n, Gate g) {
    n.tt.push_back(lut3(g.imm, n.tt[g.a], n.tt[g.b], n.tt[g.c]));
    n.g.push_back(g);
    return (int)n.tt.size() - 1;
}

// 0 if an existing signal matches, 1 if one gate suffices, 3 otherwise.
static int cost_est(const Net &n, u64 t, u64 care) {
    if (!care) return 0;
    Ref r;
    if (find_existing(n, t, care, &r)) return 0;
    Gate g;
    if (find_single(n, t, care, &g, false)) return 1;
    return 3;
}

static int g_lookahead = 0;
static Ref split_join(Net &n, u64 t, u64 care, int sel, int first_side, int depth);

static Ref solve(Net &n, u64 t, u64 care, int depth) {
    if (!care) return {-1, 0};
    Ref r;
    if (find_existing(n, t, care, &r)) return r;
    Gate g1;
    if (find_single(n, t, care, &g1, true)) return {add_gate(n, g1), 0};
    if (depth > 64) throw TooDeep();

    // choose a selector signal
    int ns = (int)n.tt.size();
    int best_sc = 1 << 30;
    std::vector<int> best;
    for (int s = 0; s < ns; s++) {
        if (restricted(s)) continue;
        u64 c1 = care & n.tt[s], c0 = care & ~n.tt[s];
        if (!c0 || !c1) continue;
        int sc = cost_est(n, t, c0) + cost_est(n, t, c1);
        if (sc < best_sc) { best_sc = sc; best.clear(); }
        if (sc == best_sc) best.push_back(s);
    }
    if (best.empty()) {
        // only restricted inputs split the care set: copy one (LUT3(i, j, j)
        // = input i) and split on the copy
        std::vector<int> cand;
        for (int i = 0; i < 6; i++)
            if (restricted(i) && (care & n.tt[i]) && (care & ~n.tt[i])) cand.push_back(i);
        if (cand.empty()) throw TooDeep();  // cannot happen for a function of the inputs
        int i = cand[rng() % cand.size()], j = (i + 1) % 6;
        while (restricted(j)) j = (j + 1) % 6;
        add_gate(n, {i, j, j, 0xF0});
        return solve(n, t, care, depth + 1);
    }
    int sel = best[rng() % best.size()];
    int first_side = (int)(rng() & 1);
    if (depth < g_lookahead && best.size() > 1) {
        // try every tied selector and both sides on copies; keep the cheapest
        size_t best_gates = (size_t)-1;
        Net best_net;
        Ref best_ref = {-1, 0};
        for (int cand : best) {
            for (int side = 0; side < 2; side++) {
                Net c = n;
                Ref r2 = split_join(c, t, care, cand, side, depth);
                if (c.g.size() < best_gates) {
                    best_gates = c.g.size();
                    best_net = c;
                    best_ref = r2;
                }
            }
        }
        n = best_net;
        return best_ref;
    }
    return split_join(n, t, care, sel, first_side, depth);
}

static Ref split_join(Net &n, u64 t, u64 care, int sel, int first_side, int depth) {
    u64 S = n.tt[sel];
    u64 care_first = care & (first_side ? S : ~S);
    u64 care_second = care & (first_side ? ~S : S);

    Ref gref = solve(n, t, care_first, depth + 1);
    u64 G = gref.idx < 0 ? 0 : (gref.neg ? ~n.tt[gref.idx] : n.tt[gref.idx]);

    // pick the join F(g, h) on the second side that leaves the easiest h
    int best_f = -1, best_fc = 1 << 30;
    u64 best_th = 0, best_ch = 0;
    int nf_tie = 0;
    for (int F = 0; F < 16; F++) {  // F bit (gv*2 + hv)
        u64 th = 0, ch = 0;
        bool ok = true;
        for (int gv = 0; gv < 2 && ok; gv++) {
            u64 pos = care_second & (gv ? G : ~G);
            if (!pos) continue;
            int f0 = (F >> (gv * 2)) & 1, f1 = (F >> (gv * 2 + 1)) & 1;
            for (int tv = 0; tv < 2; tv++) {
                u64 p = pos & (tv ? t : ~t);
                if (!p) continue;
                bool z = (f0 == tv), o = (f1 == tv);
                if (z && o) continue;          // h free here
                if (!z && !o) { ok = false; break; }
                ch |= p;
                if (o) th |= p;                // needs h = 1
            }
        }
        if (!ok) continue;
        int c = cost_est(n, th, ch);
        if (c < best_fc) { best_fc = c; best_f = F; best_th = th; best_ch = ch; nf_tie = 1; }
        else if (c == best_fc && (rng() % (++nf_tie)) == 0) { best_f = F; best_th = th; best_ch = ch; }
    }
    Ref href = solve(n, best_th, best_ch, depth + 1);
    // build the join gate LUT3(sel, g, h)
    int gi = gref.idx < 0 ? sel : gref.idx, hi = href.idx < 0 ? sel : href.idx;
    int imm = 0;
    for (int idx = 0; idx < 8; idx++) {
        int sv = (idx >> 2) & 1, gv = ((idx >> 1) & 1) ^ gref.neg, hv = (idx & 1) ^ href.neg;
        int v;
        if (sv == first_side) v = gv;
        else v = (best_f >> (gv * 2 + hv)) & 1;
        imm |= v << idx;
    }
    return {add_gate(n, {sel, gi, hi, imm}), 0};
}

// Drop gates no output depends on; renumber.
static Net prune(const Net &n) {
    int ns = (int)n.tt.size();
    std::vector<int> live(ns, 0);
    for (int q = 0; q < 4; q++) live[n.out[q].idx] = 1;
    for (int s = ns - 1; s >= 6; s--)
        if (live[s]) {
            const Gate &g = n.g[s - 6];
            live[g.a] = live[g.b] = live[g.c] = 1;
        }
    std::vector<int> map(ns, -1);
    Net m;
    for (int q = 0; q < 6; q++) { m.tt.push_back(n.tt[q]); map[q] = q; }
    for (int s = 6; s < ns; s++)
        if (live[s]) {
            Gate g = n.g[s - 6];
            g.a = map[g.a]; g.b = map[g.b]; g.c = map[g.c];
            map[s] = add_gate(m, g);
        }
    for (int q = 0; q < 4; q++) m.out[q] = {map[n.out[q].idx], n.out[q].neg};
    return m;
}

int main(int argc, char **argv) {
    if (argc != 4 + 63) {
        fprintf(stderr, "usage: %s restarts seed v0 .. v63   (env SBOX_LOOKAHEAD=depth, SBOX_RESTRICT=mask)\n", argv[0]);
        return 1;
    }
    if (getenv("SBOX_LOOKAHEAD")) g_lookahead = atoi(getenv("SBOX_LOOKAHEAD"));
    if (getenv("SBOX_RESTRICT")) g_restrict = atoi(getenv("SBOX_RESTRICT")) & 63;
    int restarts = atoi(argv[1]);
    rng.seed(strtoull(argv[2], 0, 0));
    int box[64];
    for (int i = 0; i < 64; i++) box[i] = atoi(argv[3 + i]);
    u64 target[4] = {0, 0, 0, 0};
    for (int v = 0; v < 64; v++) {
        int row = ((v >> 5) << 1) | (v & 1), col = (v >> 1) & 15;
        int val = box[row * 16 + col];
        for (int q = 0; q < 4; q++)
            if ((val >> (3 - q)) & 1) target[q] |= 1ull << v;
    }
    Net best;
    int best_n = 1 << 30;
    for (int it = 0; it < restarts; it++) {
        Net n;
        for (int q = 0; q < 6; q++) n.tt.push_back(input_tt(q));
        int order[4] = {0, 1, 2, 3};
        for (int i = 3; i > 0; i--) std::swap(order[i], order[rng() % (i + 1)]);
        try {
            for (int oi = 0; oi < 4; oi++) {
                int q = order[oi];
                n.out[q] = solve(n, target[q], ~0ull, 0);
            }
        } catch (const TooDeep &) {
            continue;
        }
        Net p = prune(n);
        for (int q = 0; q < 4; q++) {
            u64 v = p.tt[p.out[q].idx];
            if (p.out[q].neg) v = ~v;
            if (v != target[q]) { fprintf(stderr, "verification failed\n"); return 3; }
        }
        if ((int)p.g.size() < best_n) {
            best_n = (int)p.g.size();
            best = p;
            fprintf(stderr, "restart %d: %d gates\n", it, best_n);
        }
    }
    printf("gates %d\n", best_n);
    for (size_t i = 0; i < best.g.size(); i++)
        printf("g %d %d %d %d %d\n", (int)(6 + i), best.g[i].a, best.g[i].b, best.g[i].c, best.g[i].imm);
    for (int q = 0; q < 4; q++) printf("out %d %d %d\n", q, best.out[q].idx, best.out[q].neg);
    return 0;
}
