// Key masks of the bitsliced kernels in LDS: the layout (round t, S-box j
// at kBsRoundMasks * t + kBsBoxMasks * j: 4 output masks, up to 4 second-use
// masks; then the four 32-word extra groups), how a wave writes it, and the
// round runner that reads each S-box's masks TDES_BS_PIPE boxes before use.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bitslice_core.h"
#include "generated/bitslice_keys_gen.h"

namespace tdes {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef uint32_t v3u __attribute__((ext_vector_type(3)));
typedef uint32_t v2u __attribute__((ext_vector_type(2)));

constexpr bool box_ndup_fits() {
    for (int j = 0; j < 8; j++)
        if (BS_BOX_NDUP[j] < 0 || BS_BOX_NDUP[j] > 4) return false;
    return true;
}
static_assert(box_ndup_fits(), "an S-box has at most 4 second-use inputs");

#ifndef TDES_BS_PIPE
#define TDES_BS_PIPE 2  // S-boxes between a mask request and its use
#endif

// Masks of one S-box read from LDS: a uniform address, so the 8 words are
// broadcast to the wave and enter the VALU as vector operands (an
// instruction with a scalar operand is never issued together with another
// wave's).
struct LdsBoxLoad {
    // n (0..4, the box's second uses) is a compile-time constant after
    // inlining; only words that are used are read, so no read's destination
    // register is reused while the read is in flight
    template <class P>
    __device__ __forceinline__ void operator()(BsBoxMasks &m, P p, int n) const {
        // volatile keeps each read where it is issued (otherwise the reads
        // that cross the loop back edge are folded into reads at first use)
        typedef const volatile __attribute__((address_space(3))) v4u lds_v4u;
        typedef const volatile __attribute__((address_space(3))) v3u lds_v3u;
        typedef const volatile __attribute__((address_space(3))) v2u lds_v2u;
        typedef const volatile __attribute__((address_space(3))) uint32_t lds_u;
        const v4u a = *(lds_v4u *)p;
        m.o[0] = a[0]; m.o[1] = a[1]; m.o[2] = a[2]; m.o[3] = a[3];
        if (n == 4) {
            const v4u b = *(lds_v4u *)(p + 4);
            m.e[0] = b[0]; m.e[1] = b[1]; m.e[2] = b[2]; m.e[3] = b[3];
        } else if (n == 3) {
            const v3u b = *(lds_v3u *)(p + 4);
            m.e[0] = b[0]; m.e[1] = b[1]; m.e[2] = b[2];
        } else if (n == 2) {
            const v2u b = *(lds_v2u *)(p + 4);
            m.e[0] = b[0]; m.e[1] = b[1];
        } else if (n == 1) {
            m.e[0] = *(lds_u *)(p + 4);
        }
    }
};

// Runs the rounds with each S-box's masks requested TDES_BS_PIPE boxes ahead.
struct LdsPipedRounds {
    const uint32_t *km;
    BsBoxMasks pm[8];
    __device__ __forceinline__ void start() {
#pragma unroll
        for (int j = 0; j < TDES_BS_PIPE; j++) LdsBoxLoad{}(pm[j], km + kBsBoxMasks * j, BS_BOX_NDUP[j]);
    }
    template <int PH>
    __device__ __forceinline__ void round(uint32_t (&d)[32], const uint32_t (&r)[32], int t) {
        bs_round_piped<TDES_BS_PIPE>(d, r, km + kBsRoundMasks * t, km + kBsRoundMasks * (t + 1), pm,
                                     LdsBoxLoad{});
    }
    // XOR extra group g into a, 4 masks at a time with the next 4 already
    // requested (32 masks in flight at once would need 32 more registers)
    __device__ __forceinline__ void extra(int g, uint32_t (&a)[32]) const {
        typedef const volatile __attribute__((address_space(3))) v4u lds_v4u;
        const uint32_t *p = km + (g == kGroupInitY     ? kBsInitY
                                  : g == kGroupRemask16 ? kBsRemask16
                                  : g == kGroupRemask32 ? kBsRemask32
                                                        : kBsFinalX);
        v4u m[2];
        m[0] = *(lds_v4u *)p;
#pragma unroll
        for (int b = 0; b < 8; b++) {
            if (b < 7) m[(b + 1) & 1] = *(lds_v4u *)(p + 4 * b + 4);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 4; i++) a[4 * b + i] ^= m[b & 1][i];
        }
    }
};

// kBsBoxDup[4j + i] for a j known only at run time, without a memory
// lookup: column i packed into 5-bit fields of one constant (31: unused).
constexpr uint64_t dup_column(int i) {
    uint64_t c = 0;
    for (int j = 0; j < 8; j++) c |= (uint64_t)(kBsBoxDup[4 * j + i] & 31) << (5 * j);
    return c;
}
__device__ __forceinline__ int box_dup(int j, int i) {
    constexpr uint64_t kCol[4] = {dup_column(0), dup_column(1), dup_column(2), dup_column(3)};
    const int k = (int)((kCol[i] >> (5 * j)) & 31u);
    return k == 31 ? -1 : k;
}

// A lane's share of one round's 64 mask words: lane l writes slot l % 8 of
// S-box l / 8, which is bit 4j + q of the round's first key word (slot q < 4,
// output XOR masks) or bit kBsBoxDup[4j + i] of its second (slot 4 + i,
// second uses); unused slots are 0.
struct RoundMaskLane {
    uint32_t keep, sh;
    bool second;
    __device__ __forceinline__ explicit RoundMaskLane(int lane) {
        const int j = lane >> 3, sl = lane & 7;
        const int d0 = box_dup(j, 0), d1 = box_dup(j, 1), d2 = box_dup(j, 2), d3 = box_dup(j, 3);
        const int dk = sl == 4 ? d0 : sl == 5 ? d1 : sl == 6 ? d2 : d3;
        const int bit = sl < 4 ? 4 * j + sl : dk;  // -1: unused slot
        keep = bit < 0 ? 0u : ~0u;
        sh = bit < 0 ? 0u : (uint32_t)bit;
        second = sl >= 4;
    }
    // lo, hi: the round's two key words (words 2t and 2t + 1 of a direction)
    __device__ __forceinline__ uint32_t operator()(uint32_t lo, uint32_t hi) const {
        const uint32_t w = second ? hi : lo;
        return (0u - ((w >> sh) & 1u)) & keep;
    }
};

}  // namespace tdes
