// Batched 3DES-EDE ECB: many messages of uneven length, each with its own
// key schedule and direction, in one pass over the device.
//
// Work unit: a lane slice of 256 bytes (32 blocks) of one message; a
// message of n bytes has ceil(n / 256) slices.  A single-workgroup scan
// turns the descriptors into first-slice offsets (in the caller's
// workspace); then a grid of twice the resident waves strides over the
// slices, one per lane, 64 consecutive slices per wave per step.  Each lane
// finds its message (a 64-way search for the message of the wave's first
// slice, then a shuffle search over the next 64 message starts), loads its
// 256 bytes, and runs the same bitsliced core as the plain kernel, with its
// message's key masks: two mask words per round read from the device
// schedule table (cached; identical across lanes of one message) and
// expanded bit by bit with v_bfe_i32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "bitslice_core.h"
#include "internal.h"

#ifndef TDES_BATCH_MIN_WAVES
#define TDES_BATCH_MIN_WAVES 3
#endif
#ifndef TDES_BATCH_GRID_MULT
#define TDES_BATCH_GRID_MULT 2  // launched waves per resident wave slot
#endif

namespace tdes {

namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kThreads = kWave * kWavesPerBlock;
constexpr uint32_t kSlice = 256;  // bytes per lane
constexpr int kScanThreads = 1024;

// Workspace words: [0] total slices, [1] skipped messages,
// [2 + i] first slice of message i (i = 0..n; entry n = total).
constexpr int kWsHeader = 2;

// Buffer sizes a batch's message ranges are checked against.
struct BatchBounds {
    uint64_t in_bytes, out_bytes;
};

__device__ __forceinline__ uint64_t slices_of(const tdes_msg &m, size_t n_sched, BatchBounds bb,
                                              bool *bad) {
    // bitwise, not short-circuit, so that no field is read under a branch;
    // in_bytes - nbytes may wrap, but only where nbytes <= in_bytes fails
    const bool ok = (((m.nbytes | m.in_off | m.out_off) % 8) == 0) & (m.sched_idx < n_sched) &
                    (m.dir <= 1) & (m.nbytes <= bb.in_bytes) &
                    (m.in_off <= bb.in_bytes - m.nbytes) & (m.nbytes <= bb.out_bytes) &
                    (m.out_off <= bb.out_bytes - m.nbytes);
    *bad = !ok;
    return ok ? (m.nbytes + kSlice - 1) / kSlice : 0;
}

// Inclusive scan of v over the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_scan(uint64_t v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t u = __shfl_up(v, d, kWave);
        if (lane >= d) v += u;
    }
    return v;
}

// One workgroup scans the descriptors in chunks of 16 x 512: wave w owns
// descriptors w*512 .. w*512 + 511 of the chunk and walks them 64 at a time
// (coalesced loads, issued together: the index is clamped and the result
// masked so no load sits under a branch), scanning each step with shuffles
// and carrying its own running total; one barrier then gives every wave the
// totals of the waves before it, and the first slices are written
// (coalesced).  Larger batches loop over chunks, carrying the running total.
constexpr int kScanSteps = 8;  // 64-descriptor steps per wave and chunk

__global__ __launch_bounds__(kScanThreads) void batch_scan_kernel(const tdes_msg *msgs, size_t n,
                                                                 size_t n_sched, BatchBounds bb,
                                                                 uint64_t *ws,
                                                                 uint64_t *skipped_out) {
    constexpr int kWaves = kScanThreads / kWave;
    constexpr size_t kWaveMsgs = (size_t)kWave * kScanSteps;
    constexpr size_t kChunkMsgs = kWaveMsgs * kWaves;
    __shared__ uint64_t wave_tot[kWaves];
    __shared__ uint32_t wave_bad[kWaves];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    uint64_t run = 0, bad_total = 0;
    for (size_t base = 0; base < n; base += kChunkMsgs) {
        const size_t wbase = base + (size_t)w * kWaveMsgs;
        uint64_t pre[kScanSteps];  // exclusive prefix within the wave's range
        uint64_t carry = 0;
        uint32_t nbad = 0;
#pragma unroll
        for (int k = 0; k < kScanSteps; k++) {
            const size_t i = wbase + (size_t)k * kWave + lane;
            const tdes_msg m = msgs[i < n ? i : n - 1];
            bool bad = false;
            const uint64_t vi = slices_of(m, n_sched, bb, &bad);
            const uint64_t v = i < n ? vi : 0;
            nbad += (bad && i < n) ? 1u : 0u;
            const uint64_t incl = wave_scan(v, lane);
            pre[k] = carry + incl - v;
            carry += __shfl(incl, kWave - 1, kWave);
        }
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) nbad += __shfl_xor(nbad, d, kWave);
        if (lane == 0) {
            wave_tot[w] = carry;
            wave_bad[w] = nbad;
        }
        __syncthreads();
        uint64_t before = 0, tile = 0, tile_bad = 0;
        for (int k = 0; k < kWaves; k++) {
            before += k < w ? wave_tot[k] : 0;
            tile += wave_tot[k];
            tile_bad += wave_bad[k];
        }
#pragma unroll
        for (int k = 0; k < kScanSteps; k++) {
            const size_t i = wbase + (size_t)k * kWave + lane;
            if (i < n) ws[kWsHeader + i] = run + before + pre[k];
        }
        run += tile;
        bad_total += tile_bad;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ws[0] = run;
        ws[1] = bad_total;
        ws[kWsHeader + n] = run;
        if (skipped_out != nullptr) *skipped_out = bad_total;
    }
}

// Round masks expanded from a lane's own mask words.
struct LaneMasks {
    uint32_t lo, hi;  // 32 output-XOR mask bits, 16 second-use mask bits
    __device__ __forceinline__ uint32_t operator()(int i) const {
        return (uint32_t)__builtin_amdgcn_sbfe((int)(i < 32 ? lo : hi), i < 32 ? i : i - 32, 1);
    }
};
struct LaneRounds {
    const uint32_t *kw;  // this lane's 100 mask words (round t at 2t, 2t+1)
    __device__ __forceinline__ uint2 load(int t) const {
        return *reinterpret_cast<const uint2 *>(kw + 2 * t);
    }
    __device__ __forceinline__ LaneMasks masks(uint2 w) const { return LaneMasks{w.x, w.y}; }
};

// Round masks from words the whole wave shares (a wave inside one
// message): scalar loads, scalar bit extraction, scalar VALU operands.
struct WaveMasks {
    uint32_t lo, hi;
    __device__ __forceinline__ uint32_t operator()(int i) const {
        const uint32_t w = i < 32 ? lo : hi;
        return (uint32_t)(((int32_t)(w << (31 - (i < 32 ? i : i - 32)))) >> 31);
    }
};
struct WaveRounds {
    const uint32_t *kw;  // wave-uniform
    __device__ __forceinline__ uint2 load(int t) const {
        return *reinterpret_cast<const uint2 *>(kw + 2 * t);
    }
    __device__ __forceinline__ WaveMasks masks(uint2 w) const { return WaveMasks{w.x, w.y}; }
};

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(TDES_BATCH_MIN_WAVES, 8)))
void batch_bitslice_kernel(const tdes_msg *__restrict__ msgs, size_t n_msgs,
                           const uint32_t *__restrict__ sched, size_t n_sched, const uint8_t *in,
                           uint8_t *out, const uint64_t *__restrict__ ws) {
    const uint64_t total = ws[0];
    const uint64_t *first = ws + kWsHeader;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint32_t lane = threadIdx.x % kWave;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t base = ((uint64_t)blockIdx.x * kWavesPerBlock + wave) * kWave; base < total;
         base += stride) {
        // Issue priority: the message lookup, loads and input transposes at
        // the highest, the rounds at the lowest, so a wave that has just
        // started reaches its rounds sooner (measured at a settled clock:
        // 2 % faster).
        __builtin_amdgcn_s_setprio(3);
        // Message holding slice `base`: the largest m with first[m] <= base
        // (first[] is non-decreasing, first[n_msgs] = total > base).  A
        // 64-way search: each step every lane tests one evenly spaced entry
        // and a ballot keeps the sub-range, so 16k messages take 3 steps.
        size_t lo = 0, hi = n_msgs;  // first[lo] <= base < first[hi]
        while (hi - lo > 1) {
            const size_t step = (hi - lo + kWave - 1) / kWave;
            const size_t idx = lo + (size_t)(lane + 1) * step;
            const bool le = idx < hi && first[idx] <= base;
            const size_t k = (size_t)__popcll(__ballot(le));  // tests passed: a prefix of lanes
            const size_t nlo = lo + k * step, nhi = lo + (k + 1) * step;
            lo = nlo;
            hi = nhi < hi ? nhi : hi;
        }
        // Each lane's message: m0 plus the number of the next 64 message
        // starts at or before its slice, found by a binary search over the
        // starts held one per lane.  Past 63 of them (only with empty
        // messages) the lane walks on.
        const uint64_t s = base + lane;
        const bool active = s < total;
        const size_t nxt = lo + 1 + lane;
        const uint64_t start_l = nxt <= n_msgs ? first[nxt] : ~0ull;
        int r = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const uint64_t b = __shfl(start_l, r + step - 1);
            if (b <= s) r += step;
        }
        // (a lane past the end keeps m0: its count may include first[n_msgs])
        size_t m = active ? lo + (size_t)r : lo;
        if (active)
            while (first[m + 1] <= s) m++;
        const tdes_msg d = msgs[m];
        const uint64_t off = (s - first[m]) * kSlice;
        const uint32_t nb = active ? (uint32_t)min((uint64_t)kSlice, d.nbytes - off) : 0u;
        const uint8_t *src = in + d.in_off + off;
        uint8_t *dst = out + d.out_off + off;
        const uint32_t sidx = d.sched_idx < n_sched ? d.sched_idx : 0u;
        const uint32_t *kw = sched + (size_t)sidx * kDeviceScheduleWords + (d.dir & 1u) * kDirWords;

        uint32_t h0[32], h1[32];
#pragma unroll
        for (int k = 0; k < 32; k++) {
            uint2 v = make_uint2(0u, 0u);
            if ((uint32_t)k * 8u < nb) v = *reinterpret_cast<const uint2 *>(src + 8 * k);
            h0[k] = v.x;
            h1[k] = v.y;
        }
        transpose32(h0);
        transpose32(h1);
        // lane 0's schedule, addressed from the kernel argument so the
        // compiler may read it with scalar loads
        const uint32_t s0 = __builtin_amdgcn_readfirstlane(sidx);
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(d.dir & 1u);
        const uint32_t *kw0 = sched + (size_t)s0 * kDeviceScheduleWords + d0 * kDirWords;
        __builtin_amdgcn_s_setprio(0);
        if (__all(active && sidx == s0 && (d.dir & 1u) == d0)) {
            // every lane works on the same message and direction
            auto rr = prefetch_rounds(WaveRounds{kw0}, [kw0](int g, int i) {
                return (uint32_t)(((int32_t)(kw0[96 + g] << (31 - i))) >> 31);
            });
            des3_planes(h0, h1, rr);
        } else {
            auto rr = prefetch_rounds(LaneRounds{kw}, [kw](int g, int i) {
                return (uint32_t)__builtin_amdgcn_sbfe((int)kw[96 + g], i, 1);
            });
            des3_planes(h0, h1, rr);
        }
        transpose32(h0);
        transpose32(h1);
#pragma unroll
        for (int k = 0; k < 32; k++)
            if ((uint32_t)k * 8u < nb)
                *reinterpret_cast<uint2 *>(dst + 8 * k) = make_uint2(h0[k], h1[k]);
    }
}

// One thread per (bundle, direction): the three key schedules, then the
// 100 mask words of that direction.
__global__ __launch_bounds__(256) void expand_kernel(const uint8_t *keys24, size_t n,
                                                    uint32_t *schedules) {
    const size_t g = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= 2 * n) return;
    const size_t b = g / 2;
    const int dir = (int)(g % 2);
    uint8_t key[24];
    for (int i = 0; i < 24; i++) key[i] = keys24[24 * b + i];
    uint64_t k[3][16];
    for (int j = 0; j < 3; j++) des_round_keys(key + 8 * j, k[j]);
    bitslice_mask_words(k, dir, schedules + b * kDeviceScheduleWords + dir * kDirWords);
}

// The batched kernel's grid: TDES_BATCH_GRID_MULT times the workgroups that
// fit at once.  Each wave strides over the 64-slice groups, so any grid is
// correct; launching more waves than fit lets the hardware start a new wave
// wherever one finishes, so the last groups of a batch are spread over the
// whole GPU instead of being left to the persistent waves' final pass (a
// wave with no group left exits at once).
//
// The multiplier is TDES_BATCH_GRID_MULT unless tdes_batch_autotune has
// measured a better one for the current device.
constexpr int kMaxDevices = 64;
constexpr int kMaxGridMult = 4;
std::atomic<int> g_tuned_mult[kMaxDevices];  // 0: not tuned

int current_device() {
    int dev = 0;
    return hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices ? dev : 0;
}

// Workgroups of the batched kernel that fit on the current device at once,
// cached per device.
std::atomic<int> g_resident[kMaxDevices];

int resident_blocks() {
    const int dev = current_device();
    int v = g_resident[dev].load();
    if (v == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        v = cus * 4 * TDES_BATCH_MIN_WAVES / kWavesPerBlock;  // 4 SIMDs per CU
        g_resident[dev].store(v);
    }
    return v;
}

int batch_grid_blocks() {
    const int m = g_tuned_mult[current_device()].load();
    return resident_blocks() * (m > 0 ? m : TDES_BATCH_GRID_MULT);
}

}  // namespace

hipError_t launch_expand(const uint8_t *keys24, size_t n, uint32_t *schedules, hipStream_t stream) {
    const size_t threads = 2 * n, blocks = (threads + 255) / 256;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(expand_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, keys24, n,
                       schedules);
    return hipGetLastError();
}

hipError_t launch_batch_prefixed(const tdes_msg *msgs, size_t n_msgs, const uint32_t *schedules,
                                 size_t n_schedules, const uint8_t *in, uint8_t *out,
                                 const uint64_t *ws, hipStream_t stream) {
    hipLaunchKernelGGL(batch_bitslice_kernel, dim3(batch_grid_blocks()), dim3(kThreads), 0, stream,
                       msgs, n_msgs, schedules, n_schedules, in, out, ws);
    return hipGetLastError();
}

hipError_t batch_autotune(const tdes_msg *msgs, size_t n_msgs, const uint32_t *schedules,
                          size_t n_schedules, const uint8_t *in, uint64_t in_bytes, uint8_t *out,
                          uint64_t out_bytes, uint64_t *ws, hipStream_t stream, int reps,
                          int *mult_out) {
    const int dev = current_device();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    float best_ms = 0;
    int best = TDES_BATCH_GRID_MULT;
    auto run = [&]() {
        return launch_batch(msgs, n_msgs, schedules, n_schedules, in, in_bytes, out, out_bytes, ws,
                            nullptr, stream);
    };
    for (int m = 1; m <= kMaxGridMult && e == hipSuccess; m++) {
        g_tuned_mult[dev].store(m);
        e = run();  // warm
        if (e == hipSuccess) e = hipEventRecord(a, stream);
        for (int r = 0; r < reps && e == hipSuccess; r++) e = run();
        if (e == hipSuccess) e = hipEventRecord(b, stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && (m == 1 || ms < best_ms)) {
            best_ms = ms;
            best = m;
        }
    }
    g_tuned_mult[dev].store(e == hipSuccess ? best : 0);
    if (a != nullptr) (void)hipEventDestroy(a);
    if (b != nullptr) (void)hipEventDestroy(b);
    if (e == hipSuccess) *mult_out = best;
    return e;
}

size_t batch_workspace_bytes(size_t n_msgs) { return (kWsHeader + n_msgs + 1) * sizeof(uint64_t); }

hipError_t launch_batch(const tdes_msg *msgs, size_t n_msgs, const uint32_t *schedules,
                        size_t n_schedules, const uint8_t *in, uint64_t in_bytes, uint8_t *out,
                        uint64_t out_bytes, uint64_t *ws, uint64_t *skipped_out,
                        hipStream_t stream) {
    hipLaunchKernelGGL(batch_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, msgs, n_msgs,
                       n_schedules, BatchBounds{in_bytes, out_bytes}, ws, skipped_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_bitslice_kernel, dim3(batch_grid_blocks()), dim3(kThreads), 0, stream,
                       msgs, n_msgs, schedules, n_schedules, in, out, ws);
    return hipGetLastError();
}

}  // namespace tdes
