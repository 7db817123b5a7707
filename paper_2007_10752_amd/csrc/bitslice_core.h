// The bitsliced 3DES-EDE core shared by the plain and the batched kernels:
// in-lane 32x32 bit transposes and the 48 rounds on 64 plane words.
//
// Plane form: after transposing the 32 first words and the 32 second words
// of 32 blocks, plane h*32 + p holds bit position p of word h of all 32
// blocks (one block per bit).  IP, E, P and FP are then renamings of
// planes (tables in generated/bitslice_gen.h); key mixing uses 0 / ~0 masks
// (the "key-carrying" scheme described in keysched.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "generated/bitslice_gen.h"

namespace tdes {

// One swap-move stage of the 32x32 transpose: rows i and i+J (i & J == 0)
// exchange the J-bit groups where row bit J differs from column bit J.
template <int J>
__device__ __forceinline__ void swap_stage(uint32_t (&x)[32]) {
#pragma unroll
    for (int i = 0; i < 32; i++) {
        if (i & J) continue;
        const uint32_t a = x[i], b = x[i + J];
        if (J == 16) {
            x[i] = __builtin_amdgcn_perm(b, a, 0x05040100u);
            x[i + J] = __builtin_amdgcn_perm(b, a, 0x07060302u);
        } else if (J == 8) {
            x[i] = __builtin_amdgcn_perm(b, a, 0x06020400u);
            x[i + J] = __builtin_amdgcn_perm(b, a, 0x07030501u);
        } else {
            constexpr uint32_t m = J == 4 ? 0x0F0F0F0Fu : J == 2 ? 0x33333333u : 0x55555555u;
            x[i] = (a & m) | ((b << J) & ~m);
            x[i + J] = ((a >> J) & m) | (b & ~m);
        }
    }
}

// Exact transpose: afterwards bit b of x[p] is the old bit p of x[b].
__device__ __forceinline__ void transpose32(uint32_t (&x)[32]) {
    swap_stage<16>(x);
    swap_stage<8>(x);
    swap_stage<4>(x);
    swap_stage<2>(x);
    swap_stage<1>(x);
}

// The extra mask groups of a launch: initial mask of R, re-masks before
// rounds 16 and 32, final unmask of X.
enum { kGroupInitY = 0, kGroupRemask16 = 1, kGroupRemask32 = 2, kGroupFinalX = 3 };

// Round masks fetched a whole round at a time: rm.load(t) fetches what
// round t needs and rm.masks(v) turns it into the mask source bs_round reads.
// Fetches are issued two rounds ahead, so memory latency overlaps the two
// rounds before.
template <class RoundMasks>
struct PrefetchRounds {
    RoundMasks rm;
    decltype(rm.load(0)) buf[2];
    __device__ __forceinline__ void start() {
        buf[0] = rm.load(0);
        buf[1] = rm.load(1);
    }
    // PH = t % 2, known at compile time so buf stays in registers
    template <int PH>
    __device__ __forceinline__ void round(uint32_t (&d)[32], const uint32_t (&r)[32], int t) {
        const auto next = rm.load(t + 2);  // past round 47: harmless, unused
        bs_round(d, r, rm.masks(buf[PH]));
        buf[PH] = next;
    }
};

// 3DES-EDE on 32 blocks held as planes h0 (word 0) and h1 (word 1), in
// place.  rr runs the rounds: rr.start() once, then rr.round<t % 2>(d, r, t)
// for t = 0..47 (d ^= f(r, K_t)).  em(g, i) gives mask i of extra group g.
template <class RoundRunner, class ExtraMasks>
__device__ __forceinline__ void des3_planes(uint32_t (&h0)[32], uint32_t (&h1)[32],
                                            RoundRunner &rr, const ExtraMasks &em) {
    uint32_t X[32], Y[32];
#pragma unroll
    for (int i = 0; i < 32; i++) {
        X[i] = BS_IP_L[i] < 32 ? h0[BS_IP_L[i]] : h1[BS_IP_L[i] - 32];
        Y[i] = (BS_IP_R[i] < 32 ? h0[BS_IP_R[i]] : h1[BS_IP_R[i] - 32]) ^ em(kGroupInitY, i);
    }
    rr.start();
    // Pass 1 (L = X, R = Y); ends with X = L16, Y = R16.
#pragma unroll 1
    for (int r = 0; r < 16; r += 2) {
        rr.template round<0>(X, Y, r);
        rr.template round<1>(Y, X, r + 1);
    }
    // Pass 2 starts from R16 || L16 of pass 1: L = Y, R = X.
#pragma unroll
    for (int i = 0; i < 32; i++) X[i] ^= em(kGroupRemask16, i);
#pragma unroll 1
    for (int r = 16; r < 32; r += 2) {
        rr.template round<0>(Y, X, r);
        rr.template round<1>(X, Y, r + 1);
    }
    // Pass 3: L = X, R = Y again; ends with X = L16, Y = R16.
#pragma unroll
    for (int i = 0; i < 32; i++) Y[i] ^= em(kGroupRemask32, i);
#pragma unroll 1
    for (int r = 32; r < 48; r += 2) {
        rr.template round<0>(X, Y, r);
        rr.template round<1>(Y, X, r + 1);
    }
#pragma unroll
    for (int i = 0; i < 32; i++) X[i] ^= em(kGroupFinalX, i);
    // preoutput R16 || L16 = Y || X, then FP as renaming
#pragma unroll
    for (int q = 0; q < 32; q++) {
        h0[q] = BS_FP_SRC[q] < 32 ? Y[BS_FP_SRC[q]] : X[BS_FP_SRC[q] - 32];
        h1[q] = BS_FP_SRC[32 + q] < 32 ? Y[BS_FP_SRC[32 + q]] : X[BS_FP_SRC[32 + q] - 32];
    }
}

}  // namespace tdes
