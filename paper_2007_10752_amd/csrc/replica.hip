// The paper's own GPU design (Sec. IV-B, IV-C), rebuilt on gfx950 as a
// comparison point; the library's product path is the bitsliced kernel.
//
// One workgroup of 64 threads per 64-bit block, one thread per bit, bits
// held one per byte in LDS, the permutation and S-box tables read at run
// time from read-only memory, a barrier between steps, and one DES pass per
// launch: 3DES is three launches (E_K1, D_K2, E_K3), decryption being the
// same kernel with the round keys reversed on the host.  Steps per round,
// as the paper lays them out: 48 threads expand the right half and add the
// key bits; 32 threads, four per S-box, look up the S-box and each write one
// output bit; 32 threads apply the straight permutation; 32 threads XOR it
// into the left half and swap the halves.  The data stay packed in HBM (the
// paper moved one byte per bit); the kernel unpacks and packs each block.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "generated/replica_tables_gen.h"
#include "internal.h"

namespace tdes {

namespace {

constexpr int kThreads = 64;            // one per bit of a block
constexpr unsigned kMaxGrid = 1u << 20;  // workgroups; more blocks are taken in turn

__global__ __launch_bounds__(kThreads) void replica_des_pass(const uint8_t *in, uint8_t *out,
                                                             size_t nblocks, ReplicaKeyBits keys) {
    __shared__ uint8_t text[64], left[32], right[32], er[48], sb[32], pr[32];
    const int t = threadIdx.x;
    for (size_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
        // bit t of the block (DES bit 1 = most significant bit of byte 0)
        text[t] = (uint8_t)((in[8 * b + t / 8] >> (7 - t % 8)) & 1);
        __syncthreads();
        // initial permutation, then the split into halves
        const uint8_t v = text[kRepIP[t] - 1];
        if (t < 32)
            left[t] = v;
        else
            right[t - 32] = v;
        __syncthreads();
        for (int i = 0; i < 16; i++) {
            if (t < 48) er[t] = right[kRepE[t] - 1] ^ keys.k[48 * i + t];
            __syncthreads();
            if (t < 32) {
                const int g = t / 4, q = t % 4;
                const uint8_t *x = er + 6 * g;
                const int row = 2 * x[0] + x[5];
                const int col = 8 * x[1] + 4 * x[2] + 2 * x[3] + x[4];
                sb[t] = (uint8_t)((kRepS[64 * g + 16 * row + col] >> (3 - q)) & 1);
            }
            __syncthreads();
            if (t < 32) pr[t] = sb[kRepP[t] - 1];
            __syncthreads();
            if (t < 32) {
                const uint8_t nr = left[t] ^ pr[t];
                left[t] = right[t];
                right[t] = nr;
            }
            __syncthreads();
        }
        // R16 || L16, then the final permutation
        text[t] = t < 32 ? right[t] : left[t - 32];
        __syncthreads();
        const uint64_t bits = __ballot(text[kRepFP[t] - 1] != 0);
        if (t < 8) {
            uint32_t byte = 0;
            for (int k = 0; k < 8; k++) byte = byte << 1 | (uint32_t)((bits >> (8 * t + k)) & 1);
            out[8 * b + t] = (uint8_t)byte;
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_replica_pass(const ReplicaKeyBits &k, const uint8_t *in, uint8_t *out,
                               size_t nbytes, hipStream_t stream) {
    const size_t nblocks = nbytes / 8;
    const unsigned grid = nblocks < kMaxGrid ? (unsigned)nblocks : kMaxGrid;
    hipLaunchKernelGGL(replica_des_pass, dim3(grid), dim3(kThreads), 0, stream, in, out, nblocks, k);
    return hipGetLastError();
}

}  // namespace tdes
