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
//
// Modes.  ECB processes the loaded blocks.  CTR (SP 800-38A) processes
// counter blocks made in registers (the block at byte offset o holds
// ctr + o / 8, big-endian) and XORs the data into the result on the way
// out; nothing is loaded before the rounds.  CBC decryption decrypts the
// loaded blocks, then XORs each with the ciphertext block before it (the
// IV before the first), re-read after the rounds.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bitslice_core.h"
#include "lds_masks.h"
#include "generated/bitslice_keys_gen.h"
#include "internal.h"

#ifndef TDES_CTR_MIN_WAVES
#define TDES_CTR_MIN_WAVES 5  // CTR's and CBC's budget (a few spills between the passes)
#endif
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

// The 16-byte piece k of a lane (blocks 2k and 2k + 1), read after the
// rounds: one 16-byte load, or two 8-byte loads on the partial path.
template <bool WHOLE>
__device__ __forceinline__ v4u load_piece_late(__amdgpu_buffer_rsrc_t src, uint32_t lane_off, int k) {
    if (WHOLE) return __builtin_amdgcn_raw_buffer_load_b128(src, lane_off, k * 1024, 0);
    const v2u a = __builtin_amdgcn_raw_buffer_load_b64(src, lane_off, k * 1024, 0);
    const v2u b = __builtin_amdgcn_raw_buffer_load_b64(src, lane_off + 8u, k * 1024, 0);
    return v4u{a[0], a[1], b[0], b[1]};
}

// CBC decryption output: XOR each decrypted block with the ciphertext block
// before it.  Piece k's two previous blocks are the 16 bytes at 8 bytes
// before the piece: prev resource offset vbase + k * 1024.  The first block
// of the whole buffer takes the IV instead (the caller marks it with
// first_iv and gives it the out-of-range offset voff0, read as 0).
template <bool WHOLE>
__device__ __forceinline__ void cbc_store_blocks(const uint32_t (&h0)[32], const uint32_t (&h1)[32],
                                                 __amdgpu_buffer_rsrc_t prev,
                                                 __amdgpu_buffer_rsrc_t dst, uint32_t lane_off,
                                                 uint32_t voff0, uint32_t vbase, bool first_iv,
                                                 uint32_t iv0, uint32_t iv1) {
#pragma unroll
    for (int g = 0; g < 4; g++) {
        __builtin_amdgcn_sched_barrier(0);
        v4u pv[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int k = 4 * g + j;
            const uint32_t off = vbase + (uint32_t)(k * 1024);
            if (k == 0) {
                // two halves: block A's previous block (out of range where the
                // IV stands in), block B's (block A itself)
                const v2u a = __builtin_amdgcn_raw_buffer_load_b64(prev, voff0, 0, 0);
                const v2u b = __builtin_amdgcn_raw_buffer_load_b64(prev, off + 8u, 0, 0);
                pv[j] = v4u{a[0], a[1], b[0], b[1]};
            } else if (WHOLE) {
                pv[j] = __builtin_amdgcn_raw_buffer_load_b128(prev, off, 0, 0);
            } else {
                const v2u a = __builtin_amdgcn_raw_buffer_load_b64(prev, off, 0, 0);
                const v2u b = __builtin_amdgcn_raw_buffer_load_b64(prev, off + 8u, 0, 0);
                pv[j] = v4u{a[0], a[1], b[0], b[1]};
            }
        }
        if (g == 0 && first_iv) {
            pv[0][0] = iv0;
            pv[0][1] = iv1;
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int k = 4 * g + j;
            const v4u v = {h0[2 * k] ^ pv[j][0], h1[2 * k] ^ pv[j][1], h0[2 * k + 1] ^ pv[j][2],
                           h1[2 * k + 1] ^ pv[j][3]};
            if (WHOLE) {
                __builtin_amdgcn_raw_buffer_store_b128(v, dst, lane_off, k * 1024, 0);
            } else {
                __builtin_amdgcn_raw_buffer_store_b64(v2u{v[0], v[1]}, dst, lane_off, k * 1024, 0);
                __builtin_amdgcn_raw_buffer_store_b64(v2u{v[2], v[3]}, dst, lane_off + 8u, k * 1024, 0);
            }
        }
    }
}

// CTR output: XOR the lane's 32 input blocks into its 32 keystream blocks
// and store each piece as soon as it is complete, four pieces at a time (16
// registers of input in flight; each result goes straight to its store).
template <bool WHOLE>
__device__ __forceinline__ void xor_store_blocks(const uint32_t (&h0)[32], const uint32_t (&h1)[32],
                                                 __amdgpu_buffer_rsrc_t src,
                                                 __amdgpu_buffer_rsrc_t dst, uint32_t lane_off) {
#pragma unroll
    for (int g = 0; g < 4; g++) {
        __builtin_amdgcn_sched_barrier(0);
        v4u dv[4];
#pragma unroll
        for (int j = 0; j < 4; j++) dv[j] = load_piece_late<WHOLE>(src, lane_off, 4 * g + j);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int k = 4 * g + j;
            const v4u v = {h0[2 * k] ^ dv[j][0], h1[2 * k] ^ dv[j][1], h0[2 * k + 1] ^ dv[j][2],
                           h1[2 * k + 1] ^ dv[j][3]};
            if (WHOLE) {
                __builtin_amdgcn_raw_buffer_store_b128(v, dst, lane_off, k * 1024, 0);
            } else {
                __builtin_amdgcn_raw_buffer_store_b64(v2u{v[0], v[1]}, dst, lane_off, k * 1024, 0);
                __builtin_amdgcn_raw_buffer_store_b64(v2u{v[2], v[3]}, dst, lane_off + 8u, k * 1024, 0);
            }
        }
    }
}

// ECB fits 5 waves per SIMD (96 registers) at the budget of 4; the other
// modes need the 5-wave budget asked for explicitly.
template <bool VEC16, int MODE>
__global__ __launch_bounds__(kWave *kWavesPerBlock)
__attribute__((amdgpu_waves_per_eu(MODE == kModeEcb ? TDES_BS_MIN_WAVES : TDES_CTR_MIN_WAVES, 8)))
void tdes_bitslice_kernel(const uint8_t *in, uint8_t *out, size_t nbytes, BitsliceKeys keys,
                          ModeArgs mode) {
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
    if (MODE == kModeCtr) {
        if (live) {
            // counter blocks: ctr + (byte offset) / 8, as big-endian bytes,
            // so each 32-bit word (loaded little-endian) is byte-swapped
            const uint64_t c0 = mode.ctr + (base + lane_off) / 8;
#pragma unroll
            for (int k = 0; k < 16; k++) {
                const uint64_t ca = c0 + (uint64_t)(k * 128), cb = ca + 1;
                h0[2 * k] = __builtin_bswap32((uint32_t)(ca >> 32));
                h1[2 * k] = __builtin_bswap32((uint32_t)ca);
                h0[2 * k + 1] = __builtin_bswap32((uint32_t)(cb >> 32));
                h1[2 * k + 1] = __builtin_bswap32((uint32_t)cb);
            }
        }
    } else if (whole) {
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

    if (MODE == kModeCtr) {
        if (whole)
            xor_store_blocks<true>(h0, h1, src, dst, lane_off);
        else
            xor_store_blocks<false>(h0, h1, src, dst, lane_off);
        return;
    }
    if (MODE == kModeCbcDec) {
        // previous blocks: a resource from 8 bytes before the chunk (none
        // before the first chunk, whose first block takes the IV), so every
        // offset is non-negative
        const uint32_t shift = base > 0 ? 8u : 0u;
        const __amdgpu_buffer_rsrc_t prev = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(in + base - shift), 0, (int)(avail + shift), kBufferFlags);
        const bool first_iv = base == 0 && lane_off == 0;
        // lane_off + shift - 8 wraps for lane 0 of the first chunk; adding
        // k * 1024 (k >= 1) brings it back to k * 1024 - 8, and piece 0 of
        // that lane reads from an out-of-range offset instead
        const uint32_t vbase = lane_off + shift - 8u;
        const uint32_t voff0 = first_iv ? 0x40000000u : vbase;
        if (whole)
            cbc_store_blocks<true>(h0, h1, prev, dst, lane_off, voff0, vbase, first_iv, mode.iv0,
                                   mode.iv1);
        else
            cbc_store_blocks<false>(h0, h1, prev, dst, lane_off, voff0, vbase, first_iv, mode.iv0,
                                    mode.iv1);
        return;
    }
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

template <int MODE>
hipError_t launch_mode(const BitsliceKeys &k, const ModeArgs &m, const uint8_t *in, uint8_t *out,
                       size_t nbytes, hipStream_t stream) {
    const size_t chunks = (nbytes + kChunk - 1) / kChunk;
    const size_t blocks = (chunks + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    const bool vec16 = ((((uintptr_t)in) | ((uintptr_t)out)) & 15u) == 0;
    if (vec16)
        hipLaunchKernelGGL((tdes_bitslice_kernel<true, MODE>), dim3((unsigned)blocks),
                           dim3(kWave * kWavesPerBlock), 0, stream, in, out, nbytes, k, m);
    else
        hipLaunchKernelGGL((tdes_bitslice_kernel<false, MODE>), dim3((unsigned)blocks),
                           dim3(kWave * kWavesPerBlock), 0, stream, in, out, nbytes, k, m);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bitslice(const BitsliceKeys &k, const uint8_t *in, uint8_t *out,
                           size_t nbytes, hipStream_t stream) {
    return launch_mode<kModeEcb>(k, ModeArgs{}, in, out, nbytes, stream);
}

hipError_t launch_bitslice_ctr(const BitsliceKeys &k, uint64_t ctr, const uint8_t *in,
                               uint8_t *out, size_t nbytes, hipStream_t stream) {
    return launch_mode<kModeCtr>(k, ModeArgs{ctr, 0, 0}, in, out, nbytes, stream);
}

hipError_t launch_bitslice_cbc_dec(const BitsliceKeys &k, uint32_t iv0, uint32_t iv1,
                                   const uint8_t *in, uint8_t *out, size_t nbytes,
                                   hipStream_t stream) {
    return launch_mode<kModeCbcDec>(k, ModeArgs{0, iv0, iv1}, in, out, nbytes, stream);
}

}  // namespace tdes
