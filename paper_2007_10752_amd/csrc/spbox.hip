// Table-driven 3DES-EDE ECB kernel for gfx950: one 64-bit block per lane
// (up to four at a time, interleaved, in its grid-stride loop).
//
// Each round (Sec. III-B) computes f(R, K) as the XOR of eight lookups in
// combined S-box + straight-permutation tables SP_s[64] (32-bit words: the
// S-box output already moved to its P position), indexed by the six R bits
// the expansion feeds S-box s XORed with six round-key bits.  The tables
// live in LDS, replicated 32 times and interleaved so that entry e of copy c
// sits in bank c (byte 128 e + 4 c of the table): lane l reads copy l % 32,
// so a lookup is free of bank conflicts whatever the indices.  (8 tables x
// 64 entries x 32 copies x 4 B = 64 KiB per workgroup.)
//
// Key mixing: windows 1..6 of the expansion are contiguous in R (bit i of R
// at position 32 - i) and odd and even windows are disjoint, so XORing R
// once with the odd key chunks and once with the even ones keys windows
// 1..5.  Windows 0 and 7 wrap around; in R rotated left by 12 they sit at
// positions 7..12 and 11..16, and window 6 at 15..20, so one XOR of the
// rotated R keys windows 0 and 6 and another keys window 7.  Every window
// then lies at or above position 7: a right shift brings it to bits 7..12,
// and one three-input bitwise op masks it and adds the lane's copy offset,
// which makes the LDS byte address (the table's base goes into the
// instruction's offset field).  Shifts right, three-input bitwise ops and
// XORs of vector registers are the VALU instructions that issue together
// with another wave's; the mask and the copy offset are held in vector
// registers, and so are the round keys (read from LDS, where the workgroup
// copies them), so only the rotation issues alone.  The eight table words
// and the left half are folded by four three-input XORs.
//
// IP and FP run once per block as delta swaps; the three DES passes are
// fused as in the bitsliced kernel (FP then IP cancel between passes).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "generated/spbox_gen.h"
#include "internal.h"

namespace tdes {

namespace {

constexpr int kThreads = 1024;
constexpr int kCopies = 32;
constexpr int kTableWords = 8 * 64 * kCopies;
constexpr int kTableBytes = 64 * kCopies * 4;  // one S-box's table
constexpr uint32_t kIndexMask = 63u << 7;      // entry index, scaled by 128 bytes

__device__ __forceinline__ uint32_t rotl(uint32_t x, int s) {
    return __builtin_amdgcn_alignbit(x, x, 32 - s);
}

// A constant held in a vector register: the asm hides the value, so it is
// not folded back into a scalar or literal operand.
__device__ __forceinline__ uint32_t in_vgpr(uint32_t c) {
    uint32_t v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(c));
    return v;
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// One round: L ^ f(R, K).  `sp` is the LDS table base; `lane` is this
// lane's copy offset (4 (l % 32)); k = {odd chunks, even chunks, windows 0
// and 6 of the rotated half, window 7 of the rotated half}.
__device__ __forceinline__ uint32_t round_step(uint32_t L, uint32_t R, const uint8_t *sp,
                                               uint32_t lane, uint32_t mask, uint4 k) {
    const uint32_t ro = R ^ k.x, re = R ^ k.y, rr = rotl(R, 12);
    const uint32_t a06 = rr ^ k.z, a7 = rr ^ k.w;
    // (v >> sh) & mask | lane: 0xEA = (first & second) | third
    auto look = [&](int s, uint32_t v, int sh) {
        const uint32_t a = __builtin_amdgcn_bitop3_b32(v >> sh, mask, lane, 0xEA);
        return *reinterpret_cast<const uint32_t *>(sp + s * kTableBytes + a);
    };
    const uint32_t v0 = look(0, a06, 0), v1 = look(1, ro, 16), v2 = look(2, re, 12);
    const uint32_t v3 = look(3, ro, 8), v4 = look(4, re, 4), v5 = look(5, ro, 0);
    const uint32_t v6 = look(6, a06, 8), v7 = look(7, a7, 4);
    return xor3(xor3(v0, v1, v2), xor3(v3, v4, v5), xor3(v6, v7, L));
}

// The 48 rounds and FP/IP of N blocks at once (in + 8 b, stride blocks
// apart), interleaved so that one block's LDS reads wait while the others
// compute.
template <int N>
__device__ __forceinline__ void blocks(const uint8_t *in, uint8_t *out, size_t b, size_t stride,
                                       const uint8_t *sp, uint32_t lane, uint32_t mask,
                                       const uint4 *rk) {
    uint32_t X[N], Y[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
        const uint2 w = *reinterpret_cast<const uint2 *>(in + 8 * (b + i * stride));
        SP_IP(w.x, w.y, X[i], Y[i]);
    }
    // Pass 1: L = X, R = Y.
#pragma unroll 2
    for (int r = 0; r < 16; r += 2) {
#pragma unroll
        for (int i = 0; i < N; i++) X[i] = round_step(X[i], Y[i], sp, lane, mask, rk[r]);
#pragma unroll
        for (int i = 0; i < N; i++) Y[i] = round_step(Y[i], X[i], sp, lane, mask, rk[r + 1]);
    }
    // Pass 2 from R16 || L16: L = Y, R = X.
#pragma unroll 2
    for (int r = 16; r < 32; r += 2) {
#pragma unroll
        for (int i = 0; i < N; i++) Y[i] = round_step(Y[i], X[i], sp, lane, mask, rk[r]);
#pragma unroll
        for (int i = 0; i < N; i++) X[i] = round_step(X[i], Y[i], sp, lane, mask, rk[r + 1]);
    }
    // Pass 3: L = X, R = Y.
#pragma unroll 2
    for (int r = 32; r < 48; r += 2) {
#pragma unroll
        for (int i = 0; i < N; i++) X[i] = round_step(X[i], Y[i], sp, lane, mask, rk[r]);
#pragma unroll
        for (int i = 0; i < N; i++) Y[i] = round_step(Y[i], X[i], sp, lane, mask, rk[r + 1]);
    }
#pragma unroll
    for (int i = 0; i < N; i++) {
        uint32_t o0, o1;
        SP_FP(X[i], Y[i], o0, o1);  // preoutput R16 || L16 = Y || X
        *reinterpret_cast<uint2 *>(out + 8 * (b + i * stride)) = make_uint2(o0, o1);
    }
}

// `per`: lanes of each workgroup that take blocks (a multiple of 64, at most
// kThreads); all kThreads lanes fill the tables, then the others exit.
__global__ __launch_bounds__(kThreads) void tdes_spbox_kernel(const uint8_t *in, uint8_t *out,
                                                             size_t nblocks, uint32_t per,
                                                             SpboxKeys keys) {
    __shared__ __align__(16) uint32_t table[kTableWords];
    __shared__ uint4 rk[48];
    // the 512 entries x 32 copies as 16-byte chunks (8 per entry), lane i
    // writing chunks i, i + 1024, ...: each store of a wave covers 1 KiB in a
    // row, free of bank conflicts
    static_assert(kTableWords == 4 * 4 * kThreads && kCopies == 32, "table fill layout");
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int c = threadIdx.x + j * kThreads;
        const uint32_t v = SP_TABLE[c >> 3];
        reinterpret_cast<uint4 *>(table)[c] = make_uint4(v, v, v, v);
    }
    if (threadIdx.x < 48) {
        const int r = threadIdx.x;
        rk[r] = make_uint4(keys.w[r][0], keys.w[r][1], keys.w[r][2], keys.w[r][3]);
    }
    __syncthreads();
    if (threadIdx.x >= per) return;  // whole waves: per is a multiple of 64
    const uint8_t *sp = reinterpret_cast<const uint8_t *>(table);
    const uint32_t lane = (threadIdx.x % kCopies) * 4u;
    const uint32_t mask = in_vgpr(kIndexMask);

    // Grid-stride over blocks: four at a time while this thread has four,
    // then two, then one.
    const size_t stride = (size_t)gridDim.x * per;
    size_t b = (size_t)blockIdx.x * per + threadIdx.x;
    for (; b + 3 * stride < nblocks; b += 4 * stride) blocks<4>(in, out, b, stride, sp, lane, mask, rk);
    for (; b + stride < nblocks; b += 2 * stride) blocks<2>(in, out, b, stride, sp, lane, mask, rk);
    if (b < nblocks) blocks<1>(in, out, b, stride, sp, lane, mask, rk);
}

// Several messages, each with its own keys: workgroup g takes up to `per`
// blocks of the message whose workgroup range holds g (one block per
// working lane), after filling its tables and copying that message's round
// keys.  n <= 64, so one ballot over the messages' first workgroups finds
// the message: they do not decrease and the first is 0, so the lanes whose
// entry is at or before g are a prefix, and the last of them is the message
// (an empty message shares its first workgroup with the next one).
__global__ __launch_bounds__(kThreads) void tdes_spbox_multi_kernel(const SpboxMsg *msgs,
                                                                   uint32_t n,
                                                                   const SpboxKeys *keys,
                                                                   uint32_t per) {
    static_assert(kSpboxMultiMax <= 64, "one ballot covers the messages");
    __shared__ __align__(16) uint32_t table[kTableWords];
    __shared__ uint4 rk[48];
    const uint32_t g = blockIdx.x;
    const uint32_t l64 = threadIdx.x % 64;
    const bool le = l64 < n && msgs[l64].first_wg <= g;
    const uint32_t k = (uint32_t)__popcll(__ballot(le));
    const uint32_t m = k > 0 ? k - 1 : 0;  // (k is at least 1 when message 0 starts at 0)
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int c = threadIdx.x + j * kThreads;
        const uint32_t v = SP_TABLE[c >> 3];
        reinterpret_cast<uint4 *>(table)[c] = make_uint4(v, v, v, v);
    }
    if (threadIdx.x < 48)
        rk[threadIdx.x] = *reinterpret_cast<const uint4 *>(keys[m].w[threadIdx.x]);
    __syncthreads();
    if (threadIdx.x >= per) return;  // whole waves: per is a multiple of 64
    const SpboxMsg d = msgs[m];
    const uint64_t b = (uint64_t)(g - d.first_wg) * per + threadIdx.x;
    if (g >= d.first_wg && b < d.nblocks)
        blocks<1>(d.in, d.out, b, 0, reinterpret_cast<const uint8_t *>(table),
                  (threadIdx.x % kCopies) * 4u, in_vgpr(kIndexMask), rk);
}

// Workgroups that fit on the current device at once, cached per device
// (atomics: first calls from several threads may race; they all store the
// same value).
constexpr int kMaxDevices = 64;
std::atomic<int> g_resident[kMaxDevices];

int resident_workgroups() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
    int n = g_resident[dev].load();
    if (n == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        n = 2 * cus;  // 64 KiB of tables per workgroup: two fit in 160 KiB of LDS
        g_resident[dev].store(n);
    }
    return n;
}

}  // namespace

size_t spbox_one_pass_bytes() { return (size_t)resident_workgroups() * kThreads * 8; }

hipError_t launch_spbox(const SpboxKeys &k, const uint8_t *in, uint8_t *out, size_t nbytes,
                        hipStream_t stream) {
    const size_t nblocks = nbytes / 8;
    // Few blocks: fewer working lanes per workgroup and more workgroups, so
    // that the blocks spread over as many CUs as there are (one workgroup
    // each) rather than crowding a few CUs' LDS: the smallest per in 64,
    // 128, .. 1024 whose workgroups fit the CUs once.
    const size_t cus = (size_t)resident_workgroups() / 2;
    uint32_t per = 64;
    while (per < (uint32_t)kThreads && (nblocks + per - 1) / per > cus) per *= 2;
    size_t grid = (nblocks + per - 1) / per;
    // Two workgroups per resident slot: the second wave of workgroups fills
    // the slots of those that finish early.
    const size_t cap = 2 * (size_t)resident_workgroups();
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL(tdes_spbox_kernel, dim3((unsigned)grid), dim3(kThreads), 0, stream, in,
                       out, nblocks, per, k);
    return hipGetLastError();
}

uint32_t spbox_multi_lanes(const uint64_t *nblocks, size_t n) {
    const uint64_t cus = (uint64_t)resident_workgroups() / 2;
    uint32_t per = 64;
    for (; per < (uint32_t)kThreads; per *= 2) {
        uint64_t wgs = 0;
        for (size_t i = 0; i < n; i++) wgs += (nblocks[i] + per - 1) / per;
        if (wgs <= cus) break;
    }
    return per;
}

hipError_t launch_spbox_multi(const SpboxMsg *d_msgs, uint32_t n, const SpboxKeys *d_keys,
                              uint32_t per, uint32_t n_wg, hipStream_t stream) {
    if (n == 0 || n > kSpboxMultiMax || n_wg == 0 || per == 0 || per % 64 != 0 ||
        per > (uint32_t)kThreads)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(tdes_spbox_multi_kernel, dim3(n_wg), dim3(kThreads), 0, stream, d_msgs, n,
                       d_keys, per);
    return hipGetLastError();
}

}  // namespace tdes
