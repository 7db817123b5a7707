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
//   windows 1..5 sit at positions 27-4s .. 32-4s of R; odd and even windows
//   are disjoint, so one word carries the odd chunks and one the even ones;
//   windows 0 and 7 wrap around, and are read from R rotated left by 12,
//   at positions 7..12 and 11..16; window 6 is read there too, at 15..20,
//   apart from window 0, so one word carries chunks 0 and 6 and another
//   chunk 7.
void spbox_keys(const RoundSequence &seq, SpboxKeys *out) {
    for (int r = 0; r < 48; r++) {
        const uint64_t k = seq.rk[r];
        auto chunk = [k](int s) { return (uint32_t)((k >> (42 - 6 * s)) & 0x3Fu); };
        uint32_t ke = 0, ko = 0;
        for (int s = 1; s <= 5; s++) {
            if (s & 1) ko |= chunk(s) << (27 - 4 * s);
            else ke |= chunk(s) << (27 - 4 * s);
        }
        out->w[r][0] = ko;
        out->w[r][1] = ke;
        out->w[r][2] = (chunk(0) << 7) | (chunk(6) << 15);
        out->w[r][3] = chunk(7) << 11;
    }
}

}  // namespace tdes
