// Bitsliced 3DES-EDE ECB kernel for gfx950.
//
// Data layout.  One wave owns a 16 KiB chunk (2048 blocks).  Lane l loads
// the 16-byte pieces at chunk offsets l*16 + k*1024, k = 0..15, so every
// load instruction of the wave reads 1 KiB of contiguous memory, and the
// lane ends up with 32 blocks (which 32 is irrelevant in ECB: each block is
// stored back where it came from).  Two in-register 32x32 bit transposes turn
// the 32 blocks x 2 words into 64 "plane" words: plane h*32 + p holds bit
// position p of word h of all 32 blocks, one block per bit.
//
// Arithmetic.  In plane form every DES permutation is a renaming of
// registers: IP picks which planes form L and R, E picks which R words feed
// each S-box, P picks which L word each S-box output is XORed into, FP picks
// which word goes to which output plane.  The S-boxes (Sec. III-B) are
// gate networks of v_bitop3_b32 (any boolean function of three inputs),
// found by search and verified exhaustively at build time.  Key mixing is an
// XOR with all-zeros / all-ones masks (the key is uniform over the launch),
// mostly folded into the XOR that adds an S-box output into the other half:
// each half is kept XORed with the key bits its next round needs (the mask
// bookkeeping is done on the host, see keysched.cpp).  The three DES passes of EDE run back
// to back in registers: FP followed by IP is the identity, so the inner
// permutations vanish and the R16 || L16 swap between passes is a change of
// roles between the two halves.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "generated/bitslice_gen.h"
#include "generated/bitslice_keys_gen.h"
#include "internal.h"

namespace tdes {

namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr size_t kChunk = 16384;  // bytes per wave

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

template <bool VEC16>
__global__ __launch_bounds__(kWave *kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(4, 8)))
void tdes_bitslice_kernel(const uint8_t *in, uint8_t *out, size_t nbytes, BitsliceKeys keys) {
    // Expand the launch's key masks (bits) into 0 / ~0 words in LDS.  Read
    // back with a uniform address they are broadcast to every lane and enter
    // the VALU as vector operands (full issue rate; a scalar operand halves it).
    __shared__ __align__(16) uint32_t km[kBsNumMasks];
    for (int i = threadIdx.x; i < kBsNumMasks; i += kWave * kWavesPerBlock)
        km[i] = 0u - ((keys.bits[i / 32] >> (i % 32)) & 1u);
    __syncthreads();

    const size_t chunk = (size_t)blockIdx.x * kWavesPerBlock + (threadIdx.x / kWave);
    const size_t base = chunk * kChunk;
    if (base >= nbytes) return;  // wave-uniform
    const uint32_t lane_off = (threadIdx.x % kWave) * 16u;
    // bytes of this chunk that exist (16384 for every chunk but the last)
    const uint32_t avail = (uint32_t)(nbytes - base < kChunk ? nbytes - base : kChunk);
    const uint8_t *src = in + base;
    uint8_t *dst = out + base;

    uint32_t h0[32], h1[32];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const uint32_t o = lane_off + k * 1024u;
        uint2 a = make_uint2(0u, 0u), b = make_uint2(0u, 0u);
        if (VEC16 && o + 16u <= avail) {
            const uint4 v = *reinterpret_cast<const uint4 *>(src + o);
            a = make_uint2(v.x, v.y);
            b = make_uint2(v.z, v.w);
        } else {
            if (o + 8u <= avail) a = *reinterpret_cast<const uint2 *>(src + o);
            if (o + 16u <= avail) b = *reinterpret_cast<const uint2 *>(src + o + 8);
        }
        h0[2 * k] = a.x;
        h1[2 * k] = a.y;
        h0[2 * k + 1] = b.x;
        h1[2 * k + 1] = b.y;
    }
    transpose32(h0);
    transpose32(h1);

    uint32_t X[32], Y[32];
#pragma unroll
    for (int i = 0; i < 32; i++) {
        X[i] = BS_IP_L[i] < 32 ? h0[BS_IP_L[i]] : h1[BS_IP_L[i] - 32];
        Y[i] = (BS_IP_R[i] < 32 ? h0[BS_IP_R[i]] : h1[BS_IP_R[i] - 32]) ^ km[kBsInitY + i];
    }

    // Pass 1 (L = X, R = Y); ends with X = L16, Y = R16.
#pragma unroll 1
    for (int r = 0; r < 16; r += 2) {
        bs_round(X, Y, km + kBsRoundMasks * r);
        bs_round(Y, X, km + kBsRoundMasks * (r + 1));
    }
    // Pass 2 starts from R16 || L16 of pass 1: L = Y, R = X.
#pragma unroll
    for (int i = 0; i < 32; i++) X[i] ^= km[kBsRemask16 + i];
#pragma unroll 1
    for (int r = 16; r < 32; r += 2) {
        bs_round(Y, X, km + kBsRoundMasks * r);
        bs_round(X, Y, km + kBsRoundMasks * (r + 1));
    }
    // Pass 3: L = X, R = Y again; ends with X = L16, Y = R16.
#pragma unroll
    for (int i = 0; i < 32; i++) Y[i] ^= km[kBsRemask32 + i];
#pragma unroll 1
    for (int r = 32; r < 48; r += 2) {
        bs_round(X, Y, km + kBsRoundMasks * r);
        bs_round(Y, X, km + kBsRoundMasks * (r + 1));
    }
#pragma unroll
    for (int i = 0; i < 32; i++) X[i] ^= km[kBsFinalX + i];

#pragma unroll
    for (int q = 0; q < 32; q++) {
        h0[q] = BS_FP_SRC[q] < 32 ? Y[BS_FP_SRC[q]] : X[BS_FP_SRC[q] - 32];
        h1[q] = BS_FP_SRC[32 + q] < 32 ? Y[BS_FP_SRC[32 + q]] : X[BS_FP_SRC[32 + q] - 32];
    }
    transpose32(h0);
    transpose32(h1);

#pragma unroll
    for (int k = 0; k < 16; k++) {
        const uint32_t o = lane_off + k * 1024u;
        if (VEC16 && o + 16u <= avail) {
            *reinterpret_cast<uint4 *>(dst + o) =
                make_uint4(h0[2 * k], h1[2 * k], h0[2 * k + 1], h1[2 * k + 1]);
        } else {
            if (o + 8u <= avail) *reinterpret_cast<uint2 *>(dst + o) = make_uint2(h0[2 * k], h1[2 * k]);
            if (o + 16u <= avail)
                *reinterpret_cast<uint2 *>(dst + o + 8) = make_uint2(h0[2 * k + 1], h1[2 * k + 1]);
        }
    }
}

}  // namespace

hipError_t launch_bitslice(const BitsliceKeys &k, const uint8_t *in, uint8_t *out,
                           size_t nbytes, hipStream_t stream) {
    const size_t chunks = (nbytes + kChunk - 1) / kChunk;
    const size_t blocks = (chunks + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    const bool vec16 = ((((uintptr_t)in) | ((uintptr_t)out)) & 15u) == 0;
    if (vec16)
        hipLaunchKernelGGL(tdes_bitslice_kernel<true>, dim3((unsigned)blocks),
                           dim3(kWave * kWavesPerBlock), 0, stream, in, out, nbytes, k);
    else
        hipLaunchKernelGGL(tdes_bitslice_kernel<false>, dim3((unsigned)blocks),
                           dim3(kWave * kWavesPerBlock), 0, stream, in, out, nbytes, k);
    return hipGetLastError();
}

}  // namespace tdes
