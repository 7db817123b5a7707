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

// Round t of the 48 a 3DES pass applies: encryption runs E_K1, D_K2, E_K3,
// decryption D_K3, E_K2, D_K1 (Sec. III-B); a DES decryption uses the round
// keys in reverse.  k[b][i] is round key i+1 of base key b+1.
TDES_HD inline uint64_t round_key_at(const uint64_t (&k)[3][16], int dir, int t) {
    const int st = t / 16, r = t % 16;
    const int key = dir ? 2 - st : st;
    const bool rev = dir ? (st != 1) : (st == 1);
    return k[key][rev ? 15 - r : r];
}

TDES_HD inline bool bs_dest_is_x(int t) { return ((t / 16) % 2 == 0) == (t % 2 == 0); }

// The 100 mask words of direction dir for round keys k.
TDES_HD inline void bitslice_mask_words(const uint64_t (&k)[3][16], int dir, uint32_t *w) {
    for (int i = 0; i < kDirWords; i++) w[i] = 0;
    uint32_t mx = 0, my = 0;  // current mask bit of each word of X and Y
    uint64_t cur = round_key_at(k, dir, 0);
    for (int i = 0; i < 32; i++) my |= (uint32_t)((cur >> (47 - kBsPrimaryE[i])) & 1u) << i;
    w[96] = my;
    for (int t = 0; t < 48; t++) {
        const bool dx = bs_dest_is_x(t);
        uint32_t &ms = dx ? my : mx;
        uint32_t &md = dx ? mx : my;
        cur = round_key_at(k, dir, t);
        if (t == 16 || t == 32) {
            uint32_t m = 0;
            for (int i = 0; i < 32; i++) m |= (uint32_t)((cur >> (47 - kBsPrimaryE[i])) & 1u) << i;
            w[t == 16 ? 97 : 98] = ms ^ m;
            ms = m;
        }
        uint32_t dup = 0;
        for (int q = 0; q < 16; q++) {
            const int e = kBsDupE[q];
            dup |= (((ms >> kBsESrc[e]) & 1u) ^ (uint32_t)((cur >> (47 - e)) & 1u)) << q;
        }
        w[2 * t + 1] = dup;
        int next = -1;  // next round reading the half updated now
        for (int u = t + 1; u < 48 && next < 0; u++)
            if (bs_dest_is_x(u) != dx) next = u;
        uint32_t nm = 0;
        if (next >= 0) {
            const uint64_t nk = round_key_at(k, dir, next);
            for (int i = 0; i < 32; i++) nm |= (uint32_t)((nk >> (47 - kBsPrimaryE[i])) & 1u) << i;
        }
        uint32_t comp = 0;
        for (int o = 0; o < 32; o++) {
            const int i = kBsOutWord[o];
            comp |= (((md ^ nm) >> i) & 1u) << o;
        }
        w[2 * t] = comp;
        md = nm;
    }
    w[99] = mx;
}

}  // namespace tdes
