// Host check of the lane-parallel key expansion the batched path runs on the
// device: each round key computed on its own equals the sequential schedule,
// and the words formed lane by lane (one round per lane after the shared
// mask walk) equal the sequential mask words.  Built and run by
// test_keysched_core.py.
#include <cstdio>
#include <cstdint>

#include "keysched_core.h"

using namespace tdes;

int main() {
    uint64_t state = 0x3DE5C0DEull;
    auto next_byte = [&]() {
        state = state * 6364136223846793005ull + 1442695040888963407ull;
        return (uint8_t)(state >> 56);
    };
    int bad = 0, n = 0;
    for (int trial = 0; trial < 2000; trial++) {
        uint8_t key24[24];
        for (int i = 0; i < 24; i++) key24[i] = next_byte();
        if (trial == 0)
            for (int i = 0; i < 24; i++) key24[i] = 0;
        if (trial == 1)
            for (int i = 0; i < 24; i++) key24[i] = 0xFF;
        uint64_t k[3][16], rk[48];
        for (int b = 0; b < 3; b++) des_round_keys(key24 + 8 * b, k[b]);
        for (int r = 0; r < 48; r++) {  // one lane per round key
            rk[r] = des_round_key(key24 + 8 * (r / 16), r % 16);
            if (rk[r] != k[r / 16][r % 16]) bad++;
        }
        for (int dir = 0; dir < 2; dir++) {
            uint32_t want[kDirWords], got[kDirWords], P[48];
            bitslice_mask_words(k, dir, want);
            for (int t = 0; t < 48; t++) P[t] = bs_primary_mask(rk[round_key_slot(dir, t)]);
            for (int lane = 0; lane < 64; lane++) {
                uint32_t ms = 0, md = 0, nm = 0, extra[4];
                bs_mask_walk(
                    P,
                    [&](int t, uint32_t s0, uint32_t d0, uint32_t n0) {
                        if (t == lane) {
                            ms = s0;
                            md = d0;
                            nm = n0;
                        }
                    },
                    extra);
                if (lane < 48) {
                    got[2 * lane + 1] = bs_dup_word(ms, rk[round_key_slot(dir, lane)]);
                    got[2 * lane] = bs_comp_word(md, nm);
                } else if (lane < 52) {
                    got[96 + lane - 48] = extra[lane - 48];
                }
            }
            for (int i = 0; i < kDirWords; i++) bad += got[i] != want[i];
        }
        n++;
    }
    printf("%s %d bundles\n", bad ? "FAIL" : "ok", n);
    return bad ? 1 : 0;
}
