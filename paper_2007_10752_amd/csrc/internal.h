// Declarations shared by the host side of the library (not part of the ABI).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "tdes.h"

namespace tdes {

// The 48 round keys one 3DES pass applies, in application order
// (Sec. III-B equations; decryption of one DES stage = its keys reversed).
struct RoundSequence {
    uint64_t rk[48];  // 48-bit round keys, bit 1 = bit 47
};

// Kernel argument for the bitsliced kernel: the key masks of one launch
// as bits (mask i is bit i % 32 of bits[i / 32]; layout in
// generated/bitslice_keys_gen.h); the kernel expands them to 0 / ~0 words.
constexpr int kBitsliceMaskWords = 76;
struct BitsliceKeys {
    uint32_t bits[kBitsliceMaskWords];
};

// Kernel argument for the table kernel: per round, the key chunks XORed into
// the right half where the S-box windows sit (see spbox.hip).
struct SpboxKeys {
    uint32_t ke[48], ko[48], k0[48], k7[48];
};

void des_round_keys(const uint8_t key[8], uint64_t rk[16]);
void round_sequence(const tdes_schedule &ks, int dir, RoundSequence *seq);
void bitslice_keys(const RoundSequence &seq, BitsliceKeys *out);
void spbox_keys(const RoundSequence &seq, SpboxKeys *out);

// Launchers: enqueue on `stream`; return the HIP launch status.
hipError_t launch_bitslice(const BitsliceKeys &k, const uint8_t *in, uint8_t *out,
                           size_t nbytes, hipStream_t stream);
hipError_t launch_spbox(const SpboxKeys &k, const uint8_t *in, uint8_t *out, size_t nbytes,
                        hipStream_t stream);

}  // namespace tdes
