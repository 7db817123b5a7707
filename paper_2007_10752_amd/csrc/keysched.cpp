// Host-side DES key schedule (Sec. III-A) and the per-kernel key formats.
#include <string.h>

#include "generated/bitslice_keys_gen.h"
#include "generated/des_tables_gen.h"
#include "internal.h"

namespace tdes {

// Gather `nout` bits from the `nin`-bit value `in` (bit 1 = most
// significant): output bit j is input bit table[j-1].
static uint64_t gather(uint64_t in, int nin, const uint8_t *table, int nout) {
    uint64_t out = 0;
    for (int j = 0; j < nout; j++) out = (out << 1) | ((in >> (nin - table[j])) & 1u);
    return out;
}

static uint32_t rotl28(uint32_t v, int s) {
    return ((v << s) | (v >> (28 - s))) & 0x0FFFFFFFu;
}

void des_round_keys(const uint8_t key[8], uint64_t rk[16]) {
    uint64_t k = 0;
    for (int i = 0; i < 8; i++) k = (k << 8) | key[i];
    const uint64_t cd = gather(k, 64, kPC1, 56);          // parity bits dropped
    uint32_t c = (uint32_t)(cd >> 28), d = (uint32_t)(cd & 0x0FFFFFFFu);
    for (int i = 0; i < 16; i++) {
        c = rotl28(c, kShifts[i]);                         // cumulative
        d = rotl28(d, kShifts[i]);
        rk[i] = gather(((uint64_t)c << 28) | d, 56, kPC2, 48);
    }
}

// Encryption: E_K1, D_K2, E_K3.  Decryption: D_K3, E_K2, D_K1.
void round_sequence(const tdes_schedule &ks, int dir, RoundSequence *seq) {
    static const int kKey[2][3] = {{0, 1, 2}, {2, 1, 0}};
    static const int kRev[2][3] = {{0, 1, 0}, {1, 0, 1}};
    for (int st = 0; st < 3; st++) {
        const uint64_t *k = ks.k[kKey[dir][st]];
        for (int r = 0; r < 16; r++) seq->rk[16 * st + r] = k[kRev[dir][st] ? 15 - r : r];
    }
}

// The bitsliced kernel keeps each half XORed with a key mask so that key
// mixing costs no separate operation for most S-box inputs:
//   - a word of the source half carries the round-key bit of its primary
//     expansion position (the first of the one or two positions that read
//     it); its second position, if any, XORs the difference of the two bits;
//   - when a word of the destination half is updated, the XOR that adds the
//     S-box output also swaps its old mask for the one its next use as a
//     source needs (0 after its last use);
//   - the three fixed extra steps: mask R after IP, re-mask the source half
//     where a DES pass starts with a source already used by the previous
//     round (rounds 16 and 32), and unmask X at the end.
// Round t updates D from S: rounds of passes 1 and 3 alternate X^=f(Y),
// Y^=f(X); pass 2 starts from the swapped halves, Y^=f(X), X^=f(Y), ...
static bool dest_is_x(int t) { return ((t / 16) % 2 == 0) == (t % 2 == 0); }

void bitslice_keys(const RoundSequence &seq, BitsliceKeys *out) {
    memset(out, 0, sizeof *out);
    auto kbit = [&](int t, int e) { return (uint32_t)((seq.rk[t] >> (47 - e)) & 1u); };
    auto put = [&](int idx, uint32_t v) {
        if (v) out->bits[idx / 32] |= 1u << (idx % 32);
    };
    uint32_t mx[32], my[32];
    for (int i = 0; i < 32; i++) {
        mx[i] = 0;
        my[i] = kbit(0, kBsPrimaryE[i]);
        put(kBsInitY + i, my[i]);
    }
    for (int t = 0; t < 48; t++) {
        const bool dx = dest_is_x(t);
        uint32_t *ms = dx ? my : mx, *md = dx ? mx : my;
        if (t == 16 || t == 32) {
            const int base = t == 16 ? kBsRemask16 : kBsRemask32;
            for (int i = 0; i < 32; i++) {
                const uint32_t m = kbit(t, kBsPrimaryE[i]);
                put(base + i, ms[i] ^ m);
                ms[i] = m;
            }
        }
        for (int k = 0; k < 16; k++) {
            const int e = kBsDupE[k], j = kBsESrc[e];
            put(kBsRoundMasks * t + 32 + k, ms[j] ^ kbit(t, e));
        }
        int next = -1;  // next round reading the half updated now
        for (int u = t + 1; u < 48 && next < 0; u++)
            if (dest_is_x(u) != dx) next = u;
        for (int o = 0; o < 32; o++) {
            const int i = kBsOutWord[o];
            const uint32_t m = next < 0 ? 0u : kbit(next, kBsPrimaryE[i]);
            put(kBsRoundMasks * t + o, md[i] ^ m);
            md[i] = m;
        }
    }
    for (int i = 0; i < 32; i++) put(kBsFinalX + i, mx[i]);
}

static uint32_t mask_bit(const BitsliceKeys &k, int i) { return (k.bits[i / 32] >> (i % 32)) & 1u; }

void device_schedule_words(const tdes_schedule &ks, uint32_t out[kDeviceScheduleWords]) {
    memset(out, 0, kDeviceScheduleWords * sizeof(uint32_t));
    for (int dir = 0; dir < 2; dir++) {
        RoundSequence seq;
        BitsliceKeys k;
        round_sequence(ks, dir, &seq);
        bitslice_keys(seq, &k);
        uint32_t *w = out + dir * kDirWords;
        for (int t = 0; t < 48; t++)
            for (int o = 0; o < 48; o++)
                w[2 * t + o / 32] |= mask_bit(k, kBsRoundMasks * t + o) << (o % 32);
        static const int kExtra[4] = {kBsInitY, kBsRemask16, kBsRemask32, kBsFinalX};
        for (int g = 0; g < 4; g++)
            for (int i = 0; i < 32; i++) w[96 + g] |= mask_bit(k, kExtra[g] + i) << i;
    }
}

// Key chunk s (bits 6s+1..6s+6 of the round key) lines up with S-box window
// s of the right half R (bit i of R at position 32 - i):
//   windows 1..6 sit at positions 27-4s .. 32-4s of R; odd and even windows
//   are disjoint, so one word carries the odd chunks and one the even ones;
//   windows 0 and 7 wrap around, and are read from R rotated left by 7,
//   at positions 2..7 and 6..11.
void spbox_keys(const RoundSequence &seq, SpboxKeys *out) {
    for (int r = 0; r < 48; r++) {
        uint32_t ke = 0, ko = 0;
        for (int s = 1; s <= 6; s++) {
            const uint32_t ch = (uint32_t)((seq.rk[r] >> (42 - 6 * s)) & 0x3Fu);
            if (s & 1) ko |= ch << (27 - 4 * s);
            else ke |= ch << (27 - 4 * s);
        }
        out->ke[r] = ke;
        out->ko[r] = ko;
        out->k0[r] = (uint32_t)((seq.rk[r] >> 42) & 0x3Fu) << 2;
        out->k7[r] = (uint32_t)(seq.rk[r] & 0x3Fu) << 6;
    }
}

}  // namespace tdes
