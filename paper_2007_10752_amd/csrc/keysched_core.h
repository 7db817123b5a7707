// DES key schedule (Sec. III-A) and the bitsliced kernels' key masks,
// usable on the host and on the device (the batched and serving paths
// expand thousands of key bundles per launch on the GPU).
#pragma once
#include <stdint.h>

#include "generated/bitslice_keys_gen.h"
#include "generated/des_tables_gen.h"

#if defined(__HIPCC__)
#define TDES_HD __host__ __device__
#else
#define TDES_HD
#endif

namespace tdes {

// Bitsliced key masks of one 3DES pass in one direction, 100 words:
//   [2t]     bit o (0..31): mask folded into the XOR of S-box output o of
//            round t into the other half (o = 4*box + q)
//   [2t + 1] bit k (0..15): mask XORed into the k-th second-use input
//   [96..99] bit i: initial mask of R, re-masks before rounds 16 and 32,
//            final unmask of X.
// The scheme: each half is stored XORed with the key bits of its next use
// as a round's source.  A word's primary expansion position then needs no
// XOR (its key bit is already there); the other position of the 16
// duplicated words XORs the difference of the two key bits; the XOR that
// adds an S-box output into the other half also swaps that word's mask for
// its next use (0 after its last use).  Round t updates D from S; passes 1
// and 3 alternate X^=f(Y), Y^=f(X), pass 2 starts from the swapped halves
// (Y^=f(X), X^=f(Y), ...), so the source of rounds 16 and 32 was also the
// source of the round before and is re-masked first.
constexpr int kDirWords = 100;

TDES_HD inline uint64_t ks_gather(uint64_t in, int nin, const uint8_t *table, int nout) {
    uint64_t out = 0;
    // unrolled where nout is a constant: the table entries become shift counts
#pragma unroll
    for (int j = 0; j < nout; j++) out = (out << 1) | ((in >> (nin - table[j])) & 1u);
    return out;
}

TDES_HD inline uint32_t ks_rotl28(uint32_t v, int s) {
    return ((v << s) | (v >> (28 - s))) & 0x0FFFFFFFu;
}

// Round keys of one 64-bit key: PC-1 (parity bits dropped), two 28-bit
// halves rotated left cumulatively by the shift table, PC-2.  Round-key
// bit 1 is bit 47 of rk[i].
TDES_HD inline void des_round_keys(const uint8_t key[8], uint64_t rk[16]) {
    uint64_t k = 0;
    for (int i = 0; i < 8; i++) k = (k << 8) | key[i];
    const uint64_t cd = ks_gather(k, 64, kPC1, 56);
    uint32_t c = (uint32_t)(cd >> 28), d = (uint32_t)(cd & 0x0FFFFFFFu);
    for (int i = 0; i < 16; i++) {
        c = ks_rotl28(c, kShifts[i]);
        d = ks_rotl28(d, kShifts[i]);
        rk[i] = ks_gather(((uint64_t)c << 28) | d, 56, kPC2, 48);
    }
}

// Round key i (0..15) of one 64-bit key on its own, without the rounds
// before it: the halves are rotated once by the sum of the shift table
// through round i (modulo 28, a full turn).  Equals rk[i] of des_round_keys.
TDES_HD inline uint64_t des_round_key(const uint8_t key[8], int i) {
    uint64_t k = 0;
    for (int b = 0; b < 8; b++) k = (k << 8) | key[b];
    const uint64_t cd = ks_gather(k, 64, kPC1, 56);
    int s = 0;
#pragma unroll
    for (int j = 0; j < 16; j++) s += j <= i ? (int)kShifts[j] : 0;
    s %= 28;
    const uint32_t c = ks_rotl28((uint32_t)(cd >> 28), s);
    const uint32_t d = ks_rotl28((uint32_t)(cd & 0x0FFFFFFFu), s);
    return ks_gather(((uint64_t)c << 28) | d, 56, kPC2, 48);
}

// Round t of the 48 a 3DES pass applies: encryption runs E_K1, D_K2, E_K3,
// decryption D_K3, E_K2, D_K1 (Sec. III-B); a DES decryption uses the round
// keys in reverse.  Returns 16 * b + i for round key i+1 of base key b+1.
TDES_HD inline int round_key_slot(int dir, int t) {
    const int st = t / 16, r = t % 16;
    const int key = dir ? 2 - st : st;
    const bool rev = dir ? (st != 1) : (st == 1);
    return 16 * key + (rev ? 15 - r : r);
}

// k[b][i] is round key i+1 of base key b+1.
TDES_HD inline uint64_t round_key_at(const uint64_t (&k)[3][16], int dir, int t) {
    const int slot = round_key_slot(dir, t);
    return k[slot / 16][slot % 16];
}

TDES_HD inline bool bs_dest_is_x(int t) { return ((t / 16) % 2 == 0) == (t % 2 == 0); }

// Round u > t that next reads the half round t updates (-1: none).
TDES_HD inline int bs_next_reader(int t) {
    for (int u = t + 1; u < 48; u++)
        if (bs_dest_is_x(u) != bs_dest_is_x(t)) return u;
    return -1;
}

// Bit i: the key bit at the primary expansion position of half-word i.
TDES_HD inline uint32_t bs_primary_mask(uint64_t rk) {
    uint32_t m = 0;
    for (int i = 0; i < 32; i++) m |= (uint32_t)((rk >> (47 - kBsPrimaryE[i])) & 1u) << i;
    return m;
}

// Word 2t + 1: bit q is the key difference for the q-th second-use input,
// given the source half's mask ms and round key cur of round t.
TDES_HD inline uint32_t bs_dup_word(uint32_t ms, uint64_t cur) {
    uint32_t dup = 0;
    for (int q = 0; q < 16; q++) {
        const int e = kBsDupE[q];
        dup |= (((ms >> kBsESrc[e]) & 1u) ^ (uint32_t)((cur >> (47 - e)) & 1u)) << q;
    }
    return dup;
}

// Word 2t: bit o swaps the mask of the half-word S-box output o lands in,
// from md (before round t) to nm (its next use).
TDES_HD inline uint32_t bs_comp_word(uint32_t md, uint32_t nm) {
    uint32_t comp = 0;
    for (int o = 0; o < 32; o++) comp |= (((md ^ nm) >> kBsOutWord[o]) & 1u) << o;
    return comp;
}

// The masks the halves carry through the 48 rounds, from the primary masks
// P[t] of the rounds' keys: f(t, ms, md, nm) for every round (ms: mask of
// the source half when round t reads it; md, nm: mask of the destination
// half before and after round t), and the four extra words (initial mask of
// Y, re-masks before rounds 16 and 32, final mask of X).  Only this walk is
// sequential; the words of different rounds can be formed in parallel.
template <class F>
TDES_HD inline void bs_mask_walk(const uint32_t *P, F &&f, uint32_t extra[4]) {
    uint32_t mx = 0, my = P[0];  // current mask of each half
    extra[0] = my;
    // unrolled: the half each round writes and its next reader are then
    // constants, and the walk is a straight line of selects and XORs
#pragma unroll
    for (int t = 0; t < 48; t++) {
        const bool dx = bs_dest_is_x(t);
        uint32_t &ms = dx ? my : mx;
        uint32_t &md = dx ? mx : my;
        if (t == 16 || t == 32) {
            extra[t == 16 ? 1 : 2] = ms ^ P[t];
            ms = P[t];
        }
        const int next = bs_next_reader(t);
        const uint32_t nm = next >= 0 ? P[next] : 0u;
        f(t, ms, md, nm);
        md = nm;
    }
    extra[3] = mx;
}

// The 100 mask words of direction dir for round keys k.
TDES_HD inline void bitslice_mask_words(const uint64_t (&k)[3][16], int dir, uint32_t *w) {
    uint32_t P[48];
    for (int t = 0; t < 48; t++) P[t] = bs_primary_mask(round_key_at(k, dir, t));
    uint32_t extra[4];
    bs_mask_walk(
        P,
        [&](int t, uint32_t ms, uint32_t md, uint32_t nm) {
            w[2 * t + 1] = bs_dup_word(ms, round_key_at(k, dir, t));
            w[2 * t] = bs_comp_word(md, nm);
        },
        extra);
    for (int i = 0; i < 4; i++) w[96 + i] = extra[i];
}

}  // namespace tdes
