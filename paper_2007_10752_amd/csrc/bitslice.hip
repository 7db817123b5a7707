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

#include "bitslice_core.h"
#include "lds_masks.h"
#include "generated/bitslice_keys_gen.h"
#include "internal.h"

#ifndef TDES_BS_MIN_WAVES
#define TDES_BS_MIN_WAVES 4  // waves per SIMD the register budget must allow
#endif

namespace tdes {

namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr size_t kChunk = 16384;  // bytes per wave
// Buffer-resource word 3 for gfx9-family raw (unstructured) buffers.
constexpr int kBufferFlags = 0x00020000;

template <bool VEC16>
__global__ __launch_bounds__(kWave *kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(TDES_BS_MIN_WAVES, 8)))
void tdes_bitslice_kernel(const uint8_t *in, uint8_t *out, size_t nbytes, BitsliceKeys keys) {
    // Issue priority: a new wave's loads, mask expansion and transposes run
    // at the highest priority and its rounds at the lowest.  The SIMD's
    // arbiter otherwise favours the older waves, which are in their rounds,
    // so a new wave reaches its own rounds late and fewer waves are there to
    // pair instructions (measured: 6-9 % faster).
    __builtin_amdgcn_s_setprio(3);
    // the wave index is uniform within the wave; say so, so the chunk base
    // and the buffer resources below live in scalar registers
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const size_t chunk = (size_t)blockIdx.x * kWavesPerBlock + wave;
    const size_t base = chunk * kChunk;
    const bool live = base < nbytes;  // wave-uniform
    const uint32_t lane_off = (threadIdx.x % kWave) * 16u;
    // Bytes of this chunk that exist: 16384 except in the last chunk.  The
    // chunk is addressed through buffer resources sized to it, so the
    // hardware range check zero-fills loads and drops stores past the end.
    // The partial path (last chunk, or 8-byte aligned buffers) is written
    // with 8-byte accesses; the compiler may merge a lane's two loads into
    // one 16-byte load, which is still exact because the range check
    // applies per dword (odd block counts in the parity tests cover a piece
    // that straddles the end).
    const uint32_t avail = live ? (uint32_t)(nbytes - base < kChunk ? nbytes - base : kChunk) : 0u;
    const bool whole = VEC16 && avail == (uint32_t)kChunk;
    const __amdgpu_buffer_rsrc_t src =
        __builtin_amdgcn_make_buffer_rsrc((void *)(in + base), 0, (int)avail, kBufferFlags);
    const __amdgpu_buffer_rsrc_t dst =
        __builtin_amdgcn_make_buffer_rsrc((void *)(out + base), 0, (int)avail, kBufferFlags);

    // Request the chunk: its memory latency overlaps the mask expansion.
    uint32_t h0[32], h1[32];
    if (whole) {
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const v4u v = __builtin_amdgcn_raw_buffer_load_b128(src, lane_off, k * 1024, 0);
            h0[2 * k] = v[0];
            h1[2 * k] = v[1];
            h0[2 * k + 1] = v[2];
            h1[2 * k + 1] = v[3];
        }
    } else if (live) {
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const v2u a = __builtin_amdgcn_raw_buffer_load_b64(src, lane_off, k * 1024, 0);
            const v2u b = __builtin_amdgcn_raw_buffer_load_b64(src, lane_off + 8u, k * 1024, 0);
            h0[2 * k] = a[0];
            h1[2 * k] = a[1];
            h0[2 * k + 1] = b[0];
            h1[2 * k + 1] = b[1];
        }
    }

    // Expand the launch's key masks (bits) into 0 / ~0 words in LDS.  A
    // round's 64 words are one per lane: lane l is slot l % 8 of S-box l / 8,
    // slot q < 4 bit 4j + q of word 2t (output XOR masks), slot 4 + i bit
    // kBsBoxDup[4j + i] of word 2t + 1 (second uses).  Wave w builds rounds
    // w, w + 4, ...; its key words are uniform, read with scalar loads.  Past
    // the 48 rounds the pipeline requests kBsBoxMasks * TDES_BS_PIPE words
    // that are never used; they fall inside the extra groups.
    static_assert(kBsBoxMasks == 8 && kBsRoundMasks == kWave && kWavesPerBlock == 4, "mask layout");
    static_assert(kBsNumMasks - kBsInitY >= kBsBoxMasks * TDES_BS_PIPE, "mask pipeline overrun");
    __shared__ __align__(16) uint32_t km[kBsNumMasks];
    {
        const int lane = threadIdx.x % kWave;
        const RoundMaskLane rml(lane);
#pragma unroll
        for (int r = 0; r < 48 / kWavesPerBlock; r++) {
            const int t = (int)wave + kWavesPerBlock * r;
            // both words as scalars (read once per wave), then a per-lane pick
            km[kBsRoundMasks * t + lane] = rml(__builtin_amdgcn_readfirstlane(keys.w[2 * t]),
                                               __builtin_amdgcn_readfirstlane(keys.w[2 * t + 1]));
        }
        // extra group g = w, entry n = lane < 32: bit n of word 96 + g
        if (lane < 32) km[kBsInitY + 32 * wave + lane] = 0u - ((keys.w[96 + wave] >> lane) & 1u);
    }
    __syncthreads();
    if (!live) return;

    // one transpose at a time: interleaved, they hold more words live than
    // the register budget allows
    transpose32(h0);
    __builtin_amdgcn_sched_barrier(0);
    transpose32(h1);
    __builtin_amdgcn_sched_barrier(0);

    const uint32_t *kml = km;
    __builtin_amdgcn_s_setprio(0);
    LdsPipedRounds rr{kml};
    des3_planes(h0, h1, rr);
    __builtin_amdgcn_sched_barrier(0);
    transpose32(h0);
    __builtin_amdgcn_sched_barrier(0);
    transpose32(h1);

    if (whole) {
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const v4u v = {h0[2 * k], h1[2 * k], h0[2 * k + 1], h1[2 * k + 1]};
            __builtin_amdgcn_raw_buffer_store_b128(v, dst, lane_off, k * 1024, 0);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const v2u a = {h0[2 * k], h1[2 * k]}, b = {h0[2 * k + 1], h1[2 * k + 1]};
            __builtin_amdgcn_raw_buffer_store_b64(a, dst, lane_off, k * 1024, 0);
            __builtin_amdgcn_raw_buffer_store_b64(b, dst, lane_off + 8u, k * 1024, 0);
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
