// Host side of the key formats: round order per direction, bitsliced key
// masks (keysched_core.h) and the table kernel's key chunks.
#include <string.h>

#include "internal.h"

namespace tdes {

void round_sequence(const tdes_schedule &ks, int dir, RoundSequence *seq) {
    for (int t = 0; t < 48; t++) seq->rk[t] = round_key_at(ks.k, dir, t);
}

void bitslice_keys(const tdes_schedule &ks, int dir, BitsliceKeys *out) {
    bitslice_mask_words(ks.k, dir, out->w);
}

void device_schedule_words(const tdes_schedule &ks, uint32_t out[kDeviceScheduleWords]) {
    bitslice_mask_words(ks.k, 0, out);
    bitslice_mask_words(ks.k, 1, out + kDirWords);
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
