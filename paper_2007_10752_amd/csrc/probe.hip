// Microbenchmarks for the MI355X ceilings the cipher kernels are compared
// against: the issue rate of the 32-bit VALU instructions the bitsliced
// kernel is made of, the LDS read rate the table kernel depends on, and the
// HBM bandwidth of a plain copy.  Exported
// through include/tdes_probe.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tdes_probe.h"

namespace {

constexpr int kThreads = 256;
constexpr int kAcc = 16;  // independent accumulators per lane

// Each iteration issues kAcc instructions of one kind; accumulator j reads
// two others, so a sweep has kAcc-way instruction-level parallelism.
template <int OP>
__global__ __launch_bounds__(kThreads) void valu_probe_kernel(uint32_t *sink, uint32_t iters,
                                                              uint32_t smask) {
    uint32_t a[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; j++) a[j] = threadIdx.x * 0x9E3779B9u + j * 0x7F4A7C15u + blockIdx.x;
    for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
        for (int j = 0; j < kAcc; j++) {
            const uint32_t b = a[(j + 1) % kAcc], c = a[(j + 2) % kAcc];
            if (OP == TDES_PROBE_BITOP3)
                asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xe8"
                             : "=v"(a[j]) : "v"(a[j]), "v"(b), "v"(c));
            else if (OP == TDES_PROBE_XOR)
                asm volatile("v_xor_b32 %0, %1, %2" : "=v"(a[j]) : "v"(a[j]), "v"(a[(j + 3) % kAcc]));
            else if (OP == TDES_PROBE_XOR_SGPR)
                asm volatile("v_xor_b32 %0, %1, %2" : "=v"(a[j]) : "s"(smask), "v"(a[j]));
            else if (OP == TDES_PROBE_PERM)
                asm volatile("v_perm_b32 %0, %1, %2, %3" : "=v"(a[j]) : "v"(a[j]), "v"(b), "v"(c));
            else if (OP == TDES_PROBE_BFI)
                asm volatile("v_bfi_b32 %0, %1, %2, %3" : "=v"(a[j]) : "v"(a[j]), "v"(b), "v"(c));
            else if (OP == TDES_PROBE_LSHL)
                asm volatile("v_lshlrev_b32 %0, 3, %1" : "=v"(a[j]) : "v"(b));
            else if (OP == TDES_PROBE_LSHR)
                asm volatile("v_lshrrev_b32 %0, 3, %1" : "=v"(a[j]) : "v"(b));
            else if (OP == TDES_PROBE_ADD)
                asm volatile("v_add_u32 %0, %1, %2" : "=v"(a[j]) : "v"(a[j]), "v"(b));
            else
                asm volatile("v_bfe_i32 %0, %1, 4, 1" : "=v"(a[j]) : "v"(b));
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < kAcc; j++) r ^= a[j];
    sink[(size_t)blockIdx.x * kThreads + threadIdx.x] = r;
}

// LDS reads: every thread issues 16 reads per iteration (16-byte reads for
// TDES_PROBE_LDS_B128, else 4-byte), at addresses fixed per lane; the
// address register is made opaque each iteration, so every read is issued
// every iteration.  Per wave the 64 lanes read, for each of the 16 reads:
//   CONSEC: 64 consecutive words (every bank, no conflict);
//   SAMEBANK: words 64 apart (one bank: the worst case);
//   BCAST: one word (broadcast);
//   B128: 64 consecutive 16-byte pieces.
constexpr int kLdsWords = 16384;  // 64 KiB

template <int MODE>
__global__ __launch_bounds__(kThreads) void lds_probe_kernel(uint32_t *sink, uint32_t iters) {
    __shared__ __align__(16) uint32_t tab[kLdsWords];
    for (int i = threadIdx.x; i < kLdsWords; i += kThreads) tab[i] = (uint32_t)i * 0x9E3779B9u;
    __syncthreads();
    const uint32_t lane = threadIdx.x % 64, w = threadIdx.x / 64;
    // word index of read 0, and the word step between the 16 reads
    const uint32_t base = MODE == TDES_PROBE_LDS_B128       ? w * 4096 + lane * 4
                          : MODE == TDES_PROBE_LDS_CONSEC   ? w * 1024 + lane
                          : MODE == TDES_PROBE_LDS_SAMEBANK ? w * 4096 + lane * 64
                                                            : w * 1024;
    constexpr uint32_t kStep = MODE == TDES_PROBE_LDS_B128       ? 256
                               : MODE == TDES_PROBE_LDS_SAMEBANK ? 1
                                                                 : 64;
    uint32_t acc[16];
#pragma unroll
    for (int j = 0; j < 16; j++) acc[j] = 0;
    uint32_t idx = base;
    for (uint32_t i = 0; i < iters; i++) {
        asm volatile("" : "+v"(idx));
#pragma unroll
        for (int j = 0; j < 16; j++) {
            if (MODE == TDES_PROBE_LDS_B128) {
                // indexed in 16-byte units, so the read is known to be aligned
                const uint4 v = reinterpret_cast<const uint4 *>(tab)[(idx + j * kStep) / 4];
                acc[j] += v.x ^ v.y ^ v.z ^ v.w;
            } else {
                acc[j] += tab[idx + j * kStep];
            }
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 16; j++) r ^= acc[j];
    sink[(size_t)blockIdx.x * kThreads + threadIdx.x] = r;
}

__global__ __launch_bounds__(kThreads) void copy_probe_kernel(const uint4 *in, uint4 *out,
                                                              size_t n16) {
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n16; i += stride)
        out[i] = in[i];
}

}  // namespace

extern "C" {

int tdes_probe_valu(int op, uint32_t *d_sink, unsigned blocks, unsigned iters, void *stream) {
    if (d_sink == nullptr || blocks == 0 || iters == 0 || op < 0 || op > TDES_PROBE_BFE) return -1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 g(blocks), t(kThreads);
    const uint32_t m = 0x5A5A5A5Au;
    switch (op) {
    case TDES_PROBE_BITOP3: hipLaunchKernelGGL(valu_probe_kernel<TDES_PROBE_BITOP3>, g, t, 0, s, d_sink, iters, m); break;
    case TDES_PROBE_XOR: hipLaunchKernelGGL(valu_probe_kernel<TDES_PROBE_XOR>, g, t, 0, s, d_sink, iters, m); break;
    case TDES_PROBE_XOR_SGPR: hipLaunchKernelGGL(valu_probe_kernel<TDES_PROBE_XOR_SGPR>, g, t, 0, s, d_sink, iters, m); break;
    case TDES_PROBE_PERM: hipLaunchKernelGGL(valu_probe_kernel<TDES_PROBE_PERM>, g, t, 0, s, d_sink, iters, m); break;
    case TDES_PROBE_BFI: hipLaunchKernelGGL(valu_probe_kernel<TDES_PROBE_BFI>, g, t, 0, s, d_sink, iters, m); break;
    case TDES_PROBE_LSHL: hipLaunchKernelGGL(valu_probe_kernel<TDES_PROBE_LSHL>, g, t, 0, s, d_sink, iters, m); break;
    case TDES_PROBE_LSHR: hipLaunchKernelGGL(valu_probe_kernel<TDES_PROBE_LSHR>, g, t, 0, s, d_sink, iters, m); break;
    case TDES_PROBE_ADD: hipLaunchKernelGGL(valu_probe_kernel<TDES_PROBE_ADD>, g, t, 0, s, d_sink, iters, m); break;
    default: hipLaunchKernelGGL(valu_probe_kernel<TDES_PROBE_BFE>, g, t, 0, s, d_sink, iters, m); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -6;
}

int tdes_probe_lds(int mode, uint32_t *d_sink, unsigned blocks, unsigned iters, void *stream) {
    if (d_sink == nullptr || blocks == 0 || iters == 0 || mode < TDES_PROBE_LDS_CONSEC ||
        mode > TDES_PROBE_LDS_B128)
        return -1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 g(blocks), t(kThreads);
    switch (mode) {
    case TDES_PROBE_LDS_CONSEC: hipLaunchKernelGGL(lds_probe_kernel<TDES_PROBE_LDS_CONSEC>, g, t, 0, s, d_sink, iters); break;
    case TDES_PROBE_LDS_SAMEBANK: hipLaunchKernelGGL(lds_probe_kernel<TDES_PROBE_LDS_SAMEBANK>, g, t, 0, s, d_sink, iters); break;
    case TDES_PROBE_LDS_BCAST: hipLaunchKernelGGL(lds_probe_kernel<TDES_PROBE_LDS_BCAST>, g, t, 0, s, d_sink, iters); break;
    default: hipLaunchKernelGGL(lds_probe_kernel<TDES_PROBE_LDS_B128>, g, t, 0, s, d_sink, iters); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -6;
}

int tdes_probe_copy(const void *d_in, void *d_out, size_t nbytes, void *stream) {
    if (d_in == nullptr || d_out == nullptr || nbytes % 16 != 0 ||
        (((uintptr_t)d_in | (uintptr_t)d_out) & 15u) != 0)
        return -1;
    if (nbytes == 0) return 0;
    const size_t n16 = nbytes / 16;
    size_t grid = (n16 + kThreads * 4 - 1) / (kThreads * 4);
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(copy_probe_kernel, dim3((unsigned)grid), dim3(kThreads), 0,
                       static_cast<hipStream_t>(stream), static_cast<const uint4 *>(d_in),
                       static_cast<uint4 *>(d_out), n16);
    return hipGetLastError() == hipSuccess ? 0 : -6;
}

}  // extern "C"
