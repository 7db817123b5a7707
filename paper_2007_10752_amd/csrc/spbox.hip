// Table-driven 3DES-EDE ECB kernel for gfx950: one 64-bit block per lane.
//
// Each round (Sec. III-B) computes f(R, K) as the XOR of eight lookups in
// combined S-box + straight-permutation tables SP_s[64] (32-bit words: the
// S-box output already moved to its P position), indexed by the six R bits
// the expansion feeds S-box s XORed with six round-key bits.  The tables
// live in LDS, replicated 32 times and interleaved so that entry e of copy c
// sits in bank c: lane l reads copy l % 32, so a lookup is free of bank
// conflicts whatever the indices.  (8 tables x 64 entries x 32 copies x 4 B
// = 64 KiB per workgroup.)
//
// Key mixing: windows 1..6 of the expansion are contiguous in R (bit i of R
// at position 32 - i); odd and even windows are disjoint, so XORing R once
// with the odd key chunks and once with the even ones keys all six.
// Windows 0 and 7 wrap around and are read from R rotated left by 7.  IP and
// FP run once per block as rotate-and-mask code; the three DES passes are
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

__device__ __forceinline__ uint32_t rotl(uint32_t x, int s) {
    return __builtin_amdgcn_alignbit(x, x, 32 - s);
}

__device__ __forceinline__ uint32_t feistel(uint32_t R, const uint32_t *sp, uint32_t ke,
                                            uint32_t ko, uint32_t k0, uint32_t k7) {
    const uint32_t ro = R ^ ko, re = R ^ ke, rr = rotl(R, 7);
    const uint32_t a0 = rr ^ k0, a7 = rr ^ k7;
    // sp points at this lane's copy; entry v of table s is at sp[(s*64 + v) * 32]
    const uint32_t v0 = sp[(0 * 64 + ((a0 >> 2) & 63u)) * kCopies];
    const uint32_t v1 = sp[(1 * 64 + ((ro >> 23) & 63u)) * kCopies];
    const uint32_t v2 = sp[(2 * 64 + ((re >> 19) & 63u)) * kCopies];
    const uint32_t v3 = sp[(3 * 64 + ((ro >> 15) & 63u)) * kCopies];
    const uint32_t v4 = sp[(4 * 64 + ((re >> 11) & 63u)) * kCopies];
    const uint32_t v5 = sp[(5 * 64 + ((ro >> 7) & 63u)) * kCopies];
    const uint32_t v6 = sp[(6 * 64 + ((re >> 3) & 63u)) * kCopies];
    const uint32_t v7 = sp[(7 * 64 + ((a7 >> 6) & 63u)) * kCopies];
    return v0 ^ v1 ^ v2 ^ v3 ^ v4 ^ v5 ^ v6 ^ v7;
}

__global__ __launch_bounds__(kThreads) void tdes_spbox_kernel(const uint8_t *in, uint8_t *out,
                                                             size_t nblocks, SpboxKeys keys) {
    __shared__ uint32_t table[kTableWords];
    for (int i = threadIdx.x; i < kTableWords; i += kThreads) table[i] = SP_TABLE[i / kCopies];
    __syncthreads();
    const uint32_t *sp = table + (threadIdx.x % kCopies);

    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t b = (size_t)blockIdx.x * kThreads + threadIdx.x; b < nblocks; b += stride) {
        const uint2 w = *reinterpret_cast<const uint2 *>(in + 8 * b);
        uint32_t L, R;
        SP_IP(w.x, w.y, L, R);
        uint32_t X = L, Y = R;
        // Pass 1: L = X, R = Y.
#pragma unroll 2
        for (int r = 0; r < 16; r += 2) {
            X ^= feistel(Y, sp, keys.ke[r], keys.ko[r], keys.k0[r], keys.k7[r]);
            Y ^= feistel(X, sp, keys.ke[r + 1], keys.ko[r + 1], keys.k0[r + 1], keys.k7[r + 1]);
        }
        // Pass 2 from R16 || L16: L = Y, R = X.
#pragma unroll 2
        for (int r = 16; r < 32; r += 2) {
            Y ^= feistel(X, sp, keys.ke[r], keys.ko[r], keys.k0[r], keys.k7[r]);
            X ^= feistel(Y, sp, keys.ke[r + 1], keys.ko[r + 1], keys.k0[r + 1], keys.k7[r + 1]);
        }
        // Pass 3: L = X, R = Y.
#pragma unroll 2
        for (int r = 32; r < 48; r += 2) {
            X ^= feistel(Y, sp, keys.ke[r], keys.ko[r], keys.k0[r], keys.k7[r]);
            Y ^= feistel(X, sp, keys.ke[r + 1], keys.ko[r + 1], keys.k0[r + 1], keys.k7[r + 1]);
        }
        uint32_t o0, o1;
        SP_FP(X, Y, o0, o1);  // preoutput R16 || L16 = Y || X
        *reinterpret_cast<uint2 *>(out + 8 * b) = make_uint2(o0, o1);
    }
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

hipError_t launch_spbox(const SpboxKeys &k, const uint8_t *in, uint8_t *out, size_t nbytes,
                        hipStream_t stream) {
    const size_t nblocks = nbytes / 8;
    size_t grid = (nblocks + kThreads - 1) / kThreads;
    const size_t cap = (size_t)resident_workgroups();
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL(tdes_spbox_kernel, dim3((unsigned)grid), dim3(kThreads), 0, stream, in,
                       out, nblocks, k);
    return hipGetLastError();
}

}  // namespace tdes
