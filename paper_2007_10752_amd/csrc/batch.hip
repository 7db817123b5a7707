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
// 256 bytes, and runs the same bitsliced core as the plain kernel.  The key
// masks: a wave's 64 slices lie in a run of consecutive messages; the wave
// expands the masks of up to KMAX of them together, one round ahead, into a
// table in LDS (one row per message and round, in the plain kernel's
// layout), and each lane reads its own message's row with the plain
// kernel's piped LDS reads.  A wave spanning more messages takes one pass
// per group of KMAX.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <type_traits>

#include "bitslice_core.h"
#include "internal.h"
#include "lds_masks.h"

// The compiled variants of the batched cipher, X(KMAX, WAVES): KMAX
// messages per wave pass share the LDS mask table; WAVES waves per SIMD is
// the occupancy the register budget is set for (KMAX 16 does not fit 4).  The first is the default
// (with a grid of twice the resident workgroups); tdes_batch_autotune picks
// among all of them and grids of 1..4 times the resident workgroups.
#define TDES_BATCH_VARIANTS(X) X(8, 4) X(4, 4) X(8, 3) X(4, 3) X(16, 3) X(8, 5) X(4, 5)

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

// The descriptor scan over many workgroups: each tile of kTile descriptors
// is validated and scanned by its own workgroup (tile-local prefixes, the
// tile's total and bad count); then every tile adds the total of the tiles
// before it (one launch that sums them per workgroup up to kFusedTiles
// tiles; beyond, one workgroup scans the tiles' totals into offsets and a
// third launch adds them).  A single workgroup scanning all
// descriptors was bound by one CU's loads (16,384 descriptors: ~17 us).
// Workspace words past the first-slice table: T tile totals (then offsets)
// and T tile bad counts, T = ceil(n / kTile).
constexpr int kTile = kScanThreads;

__device__ __forceinline__ size_t tile_count(size_t n) { return (n + kTile - 1) / kTile; }

__global__ __launch_bounds__(kScanThreads) void batch_tile_scan_kernel(const tdes_msg *msgs, size_t n,
                                                                      size_t n_sched, BatchBounds bb,
                                                                      uint64_t *ws) {
    constexpr int kWaves = kScanThreads / kWave;
    __shared__ uint64_t wave_tot[kWaves];
    __shared__ uint32_t wave_bad[kWaves];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const size_t i = (size_t)blockIdx.x * kTile + threadIdx.x;
    const bool live = i < n;
    const tdes_msg m = msgs[live ? i : n - 1];
    bool bad = false;
    const uint64_t vi = slices_of(m, n_sched, bb, &bad);
    const uint64_t v = live ? vi : 0;
    const uint64_t incl = wave_scan(v, lane);
    const uint32_t nbad = (uint32_t)__popcll(__ballot(live && bad));
    if (lane == kWave - 1) wave_tot[w] = incl;
    if (lane == 0) wave_bad[w] = nbad;
    __syncthreads();
    uint64_t before = 0, tile = 0, tile_bad = 0;
    for (int k = 0; k < kWaves; k++) {
        before += k < w ? wave_tot[k] : 0;
        tile += wave_tot[k];
        tile_bad += wave_bad[k];
    }
    if (live) ws[kWsHeader + i] = before + incl - v;  // within the tile
    if (threadIdx.x == 0) {
        uint64_t *tiles = ws + kWsHeader + n + 1;
        tiles[blockIdx.x] = tile;
        tiles[tile_count(n) + blockIdx.x] = tile_bad;
    }
}

__global__ __launch_bounds__(kScanThreads) void batch_tile_offsets_kernel(size_t n, uint64_t *ws,
                                                                         uint64_t *skipped_out) {
    constexpr int kWaves = kScanThreads / kWave;
    __shared__ uint64_t wave_tot[kWaves];
    __shared__ uint64_t wave_bad[kWaves];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const size_t T = tile_count(n);
    uint64_t *tiles = ws + kWsHeader + n + 1;
    uint64_t run = 0, bad_total = 0;
    for (size_t base = 0; base < T; base += kScanThreads) {
        const size_t t = base + threadIdx.x;
        const uint64_t v = t < T ? tiles[t] : 0;
        const uint64_t b = t < T ? tiles[T + t] : 0;
        const uint64_t incl = wave_scan(v, lane);
        uint64_t bsum = b;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) bsum += __shfl_xor(bsum, d, kWave);
        if (lane == kWave - 1) wave_tot[w] = incl;
        if (lane == 0) wave_bad[w] = bsum;
        __syncthreads();
        uint64_t before = 0, chunk = 0, chunk_bad = 0;
        for (int k = 0; k < kWaves; k++) {
            before += k < w ? wave_tot[k] : 0;
            chunk += wave_tot[k];
            chunk_bad += wave_bad[k];
        }
        if (t < T) tiles[t] = run + before + incl - v;  // the tile's offset
        run += chunk;
        bad_total += chunk_bad;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ws[0] = run;
        ws[1] = bad_total;
        ws[kWsHeader + n] = run;
        if (skipped_out != nullptr) *skipped_out = bad_total;
    }
}

__global__ __launch_bounds__(kScanThreads) void batch_tile_add_kernel(size_t n, uint64_t *ws) {
    if (blockIdx.x == 0) return;  // the first tile's offset is 0
    const size_t i = (size_t)blockIdx.x * kTile + threadIdx.x;
    const uint64_t off = ws[kWsHeader + n + 1 + blockIdx.x];
    if (i < n) ws[kWsHeader + i] += off;
}

// Tile offsets and their addition in one launch, for batches of at most
// kFusedTiles tiles: workgroup b sums the totals of tiles 0..b-1 itself (one
// load per thread per 1024 tiles) and adds the sum to its tile's entries;
// the last workgroup also writes the batch's total and skipped count.
constexpr size_t kFusedTiles = 8192;

__device__ __forceinline__ uint64_t block_sum(uint64_t v, uint64_t *red) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
    if (lane == 0) red[w] = v;
    __syncthreads();
    uint64_t s = 0;
    for (int k = 0; k < kScanThreads / kWave; k++) s += red[k];
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(kScanThreads) void batch_tile_finish_kernel(size_t n, uint64_t *ws,
                                                                        uint64_t *skipped_out) {
    __shared__ uint64_t red[kScanThreads / kWave];
    const size_t T = tile_count(n), b = blockIdx.x;
    const uint64_t *tiles = ws + kWsHeader + n + 1;
    uint64_t part = 0;
    for (size_t t = threadIdx.x; t < b; t += kScanThreads) part += tiles[t];
    const uint64_t off = block_sum(part, red);
    const size_t i = b * kTile + threadIdx.x;
    if (i < n && off != 0) ws[kWsHeader + i] += off;
    if (b == T - 1) {
        uint64_t bad = 0;
        for (size_t t = threadIdx.x; t < T; t += kScanThreads) bad += tiles[T + t];
        bad = block_sum(bad, red);
        if (threadIdx.x == 0) {
            const uint64_t total = off + tiles[b];
            ws[0] = total;
            ws[1] = bad;
            ws[kWsHeader + n] = total;
            if (skipped_out != nullptr) *skipped_out = bad;
        }
    }
}

// Key masks of the messages a wave works on, expanded cooperatively into a
// table in LDS one round ahead of use (in place of each lane expanding its
// own 48 masks per round).  The wave's lanes hold consecutive slices, so a
// wave spans a run of consecutive messages; up to KMAX of them (a group) are
// handled per pass.  Table of one wave: 2 round buffers x KMAX rows x
// kRowWords words; a row holds one message's 64 masks of one round in the
// plain kernel's layout (box j at 8 j: output masks o[0..3], second-use
// masks e[0..3]), padded so that the rows of different messages start on
// different banks.  Per round and message the wave writes 64 words, one per
// lane (two VALU operations each), and every lane reads its own message's
// row with the piped LDS reads of the plain kernel.
constexpr int kRowWords = 68;

// The bit of a round's two key words (lo: output masks, hi: second uses) a
// lane expands: entry l of a row is slot l % 8 of S-box l / 8, an output
// mask (bit 4 j + q of lo) or a second-use mask (bit kBsBoxDup[4 j + i] of
// hi, as bit 32 + k of the pair); entries no S-box reads get bit 0.
__device__ __forceinline__ uint32_t row_entry_bit(int lane) {
    const int j = lane >> 3, sl = lane & 7;
    if (sl < 4) return (uint32_t)(4 * j + sl);
    const int k = box_dup(j, sl - 4);
    return k < 0 ? 0u : 32u + (uint32_t)k;
}

typedef __attribute__((address_space(3))) uint32_t lds_u32;

template <int KMAX, int PIPE = TDES_BS_PIPE>
struct TableRounds {
    lds_u32 *wr;          // this wave's table + lane: where this lane writes
    const lds_u32 *p0;    // this lane's row in round buffer 0 (buffer 1 follows)
    const uint32_t *sched;
    uint32_t woff;        // lanes 2j, 2j + 1: byte offset of message j's key words of round 0
    uint32_t wcur;        // lanes 2j, 2j + 1: message j's two key words of the round to build
    uint32_t sel;         // byte address (for ds_bpermute) of the lane holding this lane's word
                          // of message 0 (+ 8 j for message j)
    uint32_t bit;         // bit of that word this lane expands
    uint32_t kg;          // messages in the group (uniform, 1..KMAX)
    BsBoxMasks pm[8];

    static constexpr int kBuf = KMAX * kRowWords;  // words per round buffer

    __device__ __forceinline__ void fetch(int t) {
        wcur = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(sched) +
                                                   (woff + 8u * (uint32_t)t));
    }
    // message J's masks of the round whose words are in wcur, into buffer B.
    // Every row is written, also those of messages past the group (lanes
    // past 2 kg hold copies of the last message's words): the round body
    // must stay free of branches, or the compiler hoists all eight S-boxes'
    // mask reads to the top of the round loop and runs out of registers.
    // (sl: sel, made opaque each round so that sel + 8 j is computed here
    // and not hoisted out of the round loop, one register per message)
    template <int B, int J0>
    __device__ __forceinline__ void build_group(uint32_t sl) {
        constexpr int N = KMAX - J0 < 4 ? KMAX - J0 : 4;  // four reads in flight at a time
        uint32_t x[N];
#pragma unroll
        for (int i = 0; i < N; i++)
            x[i] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(sl + 8u * (J0 + i)), (int)wcur);
#pragma unroll
        for (int i = 0; i < N; i++)
            wr[B * kBuf + (J0 + i) * kRowWords] = (uint32_t)__builtin_amdgcn_sbfe((int)x[i], (int)bit, 1);
        if constexpr (J0 + N < KMAX) build_group<B, J0 + N>(sl);
    }
    // the masks of round t (its words in wcur) into buffer B = t % 2
    template <int B>
    __device__ __forceinline__ void build() {
        uint32_t sl = sel;
        asm volatile("" : "+v"(sl));
        build_group<B, 0>(sl);
    }
    __device__ __forceinline__ void start() {
        fetch(0);
        build<0>();
        fetch(1);
#pragma unroll
        for (int j = 0; j < PIPE; j++) LdsBoxLoad{}(pm[j], p0 + kBsBoxMasks * j, BS_BOX_NDUP[j]);
    }
    template <int PH>
    __device__ __forceinline__ void round(uint32_t (&d)[32], const uint32_t (&r)[32], int t) {
        // round t + 1's masks go to the other buffer, whose last reads (round
        // t - 1) were issued before: a wave's LDS operations run in order.
        // After round 47 this builds an unused round from the extra words,
        // into buffer 0, which the rounds no longer read.
        build<PH ^ 1>();
        fetch(t + 2);
        bs_round_piped<PIPE>(d, r, p0 + PH * kBuf, p0 + (PH ^ 1) * kBuf, pm, LdsBoxLoad{});
    }
    // XOR extra mask group g (word 96 + g of each message) into a: expanded
    // into a buffer the rounds are not using (buffer 1 between passes,
    // buffer 0 before the first round and after the last), then read 4
    // masks at a time with the next 4 requested
    __device__ __forceinline__ void extra(int g, uint32_t (&a)[32]) const {
        typedef const volatile __attribute__((address_space(3))) v4u lds_v4u;
        const int b = (g == kGroupRemask16 || g == kGroupRemask32) ? 1 : 0;
        const uint32_t l = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        // lanes 2j, 2j + 1: word 96 + g of message j (woff is even-word aligned
        // per lane pair, so both read the same word)
        const uint32_t xw = *reinterpret_cast<const uint32_t *>(
            reinterpret_cast<const char *>(sched) + ((woff & ~7u) + 4u * (96u + (uint32_t)g)));
        // (every row, all 64 entries: only entries 0..31 of this lane's row
        // are read)
#pragma unroll
        for (int j = 0; j < KMAX; j++) {
            const uint32_t x = (uint32_t)__builtin_amdgcn_ds_bpermute(8 * j, (int)xw);
            wr[b * kBuf + j * kRowWords] = (uint32_t)__builtin_amdgcn_sbfe((int)x, (int)(l & 31u), 1);
        }
        const lds_u32 *p = p0 + b * kBuf;
        v4u m[2];
        m[0] = *(lds_v4u *)p;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            if (q < 7) m[(q + 1) & 1] = *(lds_v4u *)(p + 4 * q + 4);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 4; i++) a[4 * q + i] ^= m[q & 1][i];
        }
    }
};

// A lane's slice between the lookup and the cipher phases of a pass: kept in
// LDS (volatile, so the compiler cannot forward it in registers), so that
// nothing of the lookup stays in registers through the rounds.
// The lanes of a wave that hold slices of one message form a run; the run
// reads and writes its message's bytes together, coalesced: lane i of a run
// of L lanes takes the 16-byte pieces at i * 16 + k * 16 L (k = 0..15) of
// the run's bytes, as the plain kernel does with a whole wave (one key per
// run, so any assignment of the run's blocks to its lanes is ECB).
struct LaneSlice {
    uint64_t src, dst;  // device addresses of the lane's run (its message's bytes in this wave)
    uint32_t nb;        // bytes of the run (0: no work for this lane)
    uint32_t row;       // this lane's row of the mask table
    uint32_t pos;       // byte offset of this lane's first piece in the run: 16 i
    uint32_t stride;    // bytes between its pieces: 16 L
};
typedef __attribute__((address_space(3))) volatile uint64_t lds_vu64;
typedef __attribute__((address_space(3))) volatile uint32_t lds_vu32;
// Global-memory views of a lane's slice (its addresses come through LDS as
// integers): 16-byte accesses at 8-byte alignment (message offsets are only
// multiples of 8) and 8-byte accesses.
typedef uint32_t v4u_a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef __attribute__((address_space(1))) const v4u_a8 g_cu4;
typedef __attribute__((address_space(1))) v4u_a8 g_u4;
typedef __attribute__((address_space(1))) const v2u g_cu2;
typedef __attribute__((address_space(1))) v2u g_u2;

// Messages per mask-table group for a wave spanning n messages: a table of
// 4 rows if they fit, else of KMAX rows (one pass if they fit; a
// table builds every one of its rows each round, so fewer rows cost less),
// else KMAX rows and one pass per KMAX messages.  Most waves of a batch of
// kilobyte messages span 2 to 5 of them.
#ifndef TDES_BATCH_ADAPT
#define TDES_BATCH_ADAPT 1
#endif
template <int KMAX>
__device__ __forceinline__ uint32_t group_rows(uint32_t n) {
    if (TDES_BATCH_ADAPT && KMAX > 4 && n <= 4) return 4;
    return KMAX;
}

template <int KMAX, int WAVES>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
void batch_bitslice_kernel(const tdes_msg *__restrict__ msgs, uint32_t n_msgs,
                           const uint32_t *__restrict__ sched, uint32_t n_sched, const uint8_t *in,
                           uint8_t *out, const uint64_t *__restrict__ ws) {
    __shared__ __align__(16) uint32_t tables[kWavesPerBlock][2 * KMAX * kRowWords];
    __shared__ LaneSlice slices[kWavesPerBlock][kWave];
    const uint64_t total = ws[0];
    const uint64_t *first = ws + kWsHeader;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint32_t lane = threadIdx.x % kWave;
    LaneSlice *mine_ls = &slices[wave][lane];
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t base = ((uint64_t)blockIdx.x * kWavesPerBlock + wave) * kWave; base < total;
         base += stride) {
        // Passes over groups of G consecutive messages of the wave: one pass
        // unless the wave's 64 slices span more than KMAX messages.
        uint32_t g0 = 0, n_wave_msgs = 1, G = KMAX;
        do {
            // Issue priority: the message lookup, loads and input transposes
            // at the highest, the rounds at the lowest, so a wave that has
            // just started reaches its rounds sooner.
            __builtin_amdgcn_s_setprio(3);
            uint32_t lo, woff;
            {
                // Message holding slice `base`: the largest m with first[m]
                // <= base (first[] is non-decreasing, first[n_msgs] = total >
                // base).  A 64-way search: each step every lane tests one
                // evenly spaced entry and a ballot keeps the sub-range, so
                // 16k messages take 3 steps.
                lo = 0;
                uint32_t hi = n_msgs;  // first[lo] <= base < first[hi]
                while (hi - lo > 1) {
                    const uint32_t step = (hi - lo + kWave - 1) / kWave;
                    const uint64_t idx = lo + (uint64_t)(lane + 1) * step;
                    const bool le = idx < hi && first[idx] <= base;
                    const uint32_t k = (uint32_t)__popcll(__ballot(le));  // a prefix of lanes
                    const uint64_t nhi = lo + (uint64_t)(k + 1) * step;
                    lo = lo + k * step;
                    hi = nhi < hi ? (uint32_t)nhi : hi;
                }
                lo = __builtin_amdgcn_readfirstlane(lo);
                // Each lane's message: m0 plus the number of the next 64
                // message starts at or before its slice, found by a binary
                // search over the starts held one per lane.  Past 63 of them
                // (only with empty messages) the lane walks on.
                const uint64_t s = base + lane;
                const bool active = s < total;
                const uint32_t nxt = lo + 1 + lane;
                const uint64_t start_l = nxt <= n_msgs ? first[nxt] : ~0ull;
                int r = 0;
#pragma unroll
                for (int step = 32; step >= 1; step >>= 1) {
                    const uint64_t b = __shfl(start_l, r + step - 1);
                    if (b <= s) r += step;
                }
                // (a lane past the end keeps m0: its count may include first[n_msgs])
                uint32_t m = active ? lo + (uint32_t)r : lo;
                if (active)
                    while (first[m + 1] <= s) m++;
                // The wave's messages lo .. m_hi (lane 0 holds the first, the
                // last active lane the last); this lane's is number m - lo.
                const uint64_t left = total - base;
                const int last = left > (uint64_t)kWave ? kWave - 1 : (int)left - 1;
                n_wave_msgs = (uint32_t)__builtin_amdgcn_readlane((int)m, last) - lo + 1;
                G = group_rows<KMAX>(n_wave_msgs);
                const uint32_t slot = m - lo;
                const bool mine = active && slot - g0 < G;
                const tdes_msg d = msgs[m];
                // this lane's run: the slices of message m in this wave
                const uint64_t f0 = first[m], f1 = first[m + 1];
                const uint64_t run0 = f0 > base ? f0 : base;
                const uint64_t run1 = f1 < base + kWave ? f1 : base + kWave;
                const uint64_t run_off = (run0 - f0) * kSlice;  // in the message
                const uint64_t run_len = (run1 - run0) * kSlice;
                const uint64_t rem = d.nbytes - run_off;
                *(lds_vu64 *)&mine_ls->src = (uint64_t)(uintptr_t)(in + d.in_off + run_off);
                *(lds_vu64 *)&mine_ls->dst = (uint64_t)(uintptr_t)(out + d.out_off + run_off);
                *(lds_vu32 *)&mine_ls->nb = mine ? (uint32_t)(rem < run_len ? rem : run_len) : 0u;
                *(lds_vu32 *)&mine_ls->pos = (uint32_t)(s - run0) * 16u;
                *(lds_vu32 *)&mine_ls->stride = (uint32_t)(run1 - run0) * 16u;
                *(lds_vu32 *)&mine_ls->row = (slot - g0) & (G - 1);  // (any row for other groups)
                // lanes 2j, 2j + 1: the two key words of round 0 of the
                // group's message j (the last one for lanes past the group)
                const uint32_t kg = min(n_wave_msgs - g0, G);
                const tdes_msg dj = msgs[lo + g0 + min(lane >> 1, kg - 1)];
                woff = 4u * ((dj.sched_idx < n_sched ? dj.sched_idx : 0u) *
                                 (uint32_t)kDeviceScheduleWords +
                             (dj.dir & 1u) * (uint32_t)kDirWords + (lane & 1u));
                if (__ballot(mine) == 0) continue;  // a group of empty messages
            }
            // load, transposes, the 48 rounds with a table of K rows (K
            // uniform over the wave), transposes, store: one copy per table
            // size, so that nothing but a few scalars is live across the choice
            auto cipher = [&](auto k_rows) {
                constexpr int K = decltype(k_rows)::value;
                uint32_t h0[32], h1[32];
                {
                    // the run's piece k for this lane, at min(pos + k stride,
                    // nb - 16): pieces past the run's last block repeat its
                    // last pieces and are written back to the same place
                    // with the same (deterministic) result, so no access
                    // leaves the run and none needs a branch
                    const uint64_t src = *(lds_vu64 *)&mine_ls->src;
                    const uint32_t nb = *(lds_vu32 *)&mine_ls->nb;
                    const uint32_t pos = *(lds_vu32 *)&mine_ls->pos;
                    const uint32_t stride = *(lds_vu32 *)&mine_ls->stride;
#pragma unroll
                    for (int k = 0; k < 32; k++) h0[k] = h1[k] = 0;
                    if (nb >= 16) {
#pragma unroll
                        for (int k = 0; k < 16; k++) {
                            const uint32_t o = min(pos + (uint32_t)k * stride, nb - 16u);
                            const v4u v = *(g_cu4 *)(uintptr_t)(src + o);
                            h0[2 * k] = v[0];
                            h1[2 * k] = v[1];
                            h0[2 * k + 1] = v[2];
                            h1[2 * k + 1] = v[3];
                        }
                    } else if (nb == 8) {  // a run of one block
                        const v2u v = *(g_cu2 *)(uintptr_t)src;
                        h0[0] = v[0];
                        h1[0] = v[1];
                    }
                }
                TableRounds<K, (WAVES >= 5 ? 1 : TDES_BS_PIPE)> rr;
                rr.kg = min(n_wave_msgs - g0, (uint32_t)K);
                rr.sched = sched;
                rr.woff = woff;
                {
                    // entry `lane` of a row: bit eb of the round's word pair
                    // (lo, hi as bits 32..63), found in lane 2j (lo) or 2j + 1 (hi)
                    const uint32_t eb = row_entry_bit((int)lane);
                    rr.sel = 4u * (eb >> 5);
                    rr.bit = eb & 31u;
                }
                rr.wr = (lds_u32 *)tables[wave] + lane;
                rr.p0 = (const lds_u32 *)tables[wave] + *(lds_vu32 *)&mine_ls->row * kRowWords;
                transpose32(h0);
                __builtin_amdgcn_sched_barrier(0);
                transpose32(h1);
                pin_words(h0);
                pin_words(h1);
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_setprio(0);
                des3_planes(h0, h1, rr);
                __builtin_amdgcn_sched_barrier(0);
                transpose32(h0);
                __builtin_amdgcn_sched_barrier(0);
                transpose32(h1);
                pin_words(h0);
                pin_words(h1);
                {
                    const uint64_t dst = *(lds_vu64 *)&mine_ls->dst;
                    const uint32_t nb = *(lds_vu32 *)&mine_ls->nb;
                    const uint32_t pos = *(lds_vu32 *)&mine_ls->pos;
                    const uint32_t stride = *(lds_vu32 *)&mine_ls->stride;
                    if (nb >= 16) {
#pragma unroll
                        for (int k = 0; k < 16; k++) {
                            const uint32_t o = min(pos + (uint32_t)k * stride, nb - 16u);
                            *(g_u4 *)(uintptr_t)(dst + o) =
                                v4u_a8{h0[2 * k], h1[2 * k], h0[2 * k + 1], h1[2 * k + 1]};
                        }
                    } else if (nb == 8) {
                        *(g_u2 *)(uintptr_t)dst = v2u{h0[0], h1[0]};
                    }
                }
            };
            if (KMAX > 4 && G == 4)
                cipher(std::integral_constant<int, (KMAX > 4 ? 4 : KMAX)>{});
            else
                cipher(std::integral_constant<int, KMAX>{});
        } while ((g0 += G) < n_wave_msgs);
    }
}

// Key expansion, one wave per bundle (four per workgroup), both directions.
// The rounds are independent once each round key is computed on its own
// (des_round_key), so lanes 0..47 each make one of the 48 round keys, then
// the primary mask of one round per direction; the mask walk that links the
// rounds is short and runs on every lane alike; lane t then forms the two
// words of round t and lanes 48..51 the four extra words.  A wave finishes
// in a few microseconds, so small batches (a request server's) do not wait
// on one thread working through a whole bundle.
constexpr int kExpandWaves = 4;

__global__ __launch_bounds__(kExpandWaves * kWave) void expand_kernel(const uint8_t *keys24,
                                                                      size_t n,
                                                                      uint32_t *schedules) {
    __shared__ uint64_t rk_s[kExpandWaves][48];
    __shared__ uint32_t p_s[kExpandWaves][2][48];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const size_t b = (size_t)blockIdx.x * kExpandWaves + w;
    const bool live = b < n;  // uniform per wave; every wave reaches the barriers
    if (live && lane < 48) {
        const uint8_t *kp = keys24 + 24 * b + 8 * (lane / 16);
        uint8_t key[8];
        for (int i = 0; i < 8; i++) key[i] = kp[i];
        rk_s[w][lane] = des_round_key(key, lane % 16);
    }
    __syncthreads();
    if (live && lane < 48)
        for (int dir = 0; dir < 2; dir++)
            p_s[w][dir][lane] = bs_primary_mask(rk_s[w][round_key_slot(dir, lane)]);
    __syncthreads();
    if (!live) return;
    for (int dir = 0; dir < 2; dir++) {
        uint32_t ms = 0, md = 0, nm = 0, extra[4];
        bs_mask_walk(
            p_s[w][dir],
            [&](int t, uint32_t s0, uint32_t d0, uint32_t n0) {
                if (t == lane) {
                    ms = s0;
                    md = d0;
                    nm = n0;
                }
            },
            extra);
        uint32_t *out = schedules + b * kDeviceScheduleWords + dir * kDirWords;
        if (lane < 48) {
            out[2 * lane + 1] = bs_dup_word(ms, rk_s[w][round_key_slot(dir, lane)]);
            out[2 * lane] = bs_comp_word(md, nm);
        } else if (lane < 52) {
            const int i = lane - 48;
            out[96 + i] = i == 0 ? extra[0] : i == 1 ? extra[1] : i == 2 ? extra[2] : extra[3];
        }
    }
}

// The batched kernel's grid: grid_mult times the workgroups that fit at
// once.  Each wave strides over the 64-slice groups, so any grid is
// correct; launching more waves than fit lets the hardware start a new wave
// wherever one finishes, so the last groups of a batch are spread over the
// whole GPU instead of being left to the persistent waves' final pass (a
// wave with no group left exits at once).
constexpr int kMaxDevices = 64;
constexpr int kMaxGridMult = 4;
constexpr BatchConfig kDefaultConfig{8, 4, 2};

int current_device() {
    int dev = 0;
    return hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices ? dev : 0;
}

// Workgroups of variant <K, W> that fit on the current device at once
// (occupancy calculator: registers and LDS), cached per device.
template <int K, int W>
int resident_blocks() {
    static std::atomic<int> cache[kMaxDevices];
    const int dev = current_device();
    int v = cache[dev].load();
    if (v == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_bitslice_kernel<K, W>,
                                                         kThreads, 0) != hipSuccess ||
            per_cu <= 0)
            per_cu = W;  // 4 SIMDs x W waves, 4 waves per workgroup
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        v = per_cu * cus;
        cache[dev].store(v);
    }
    return v;
}

// (max_blocks: when the host knows the batch's slices, no more workgroups
// than they fill; 0 = unknown)
template <int K, int W>
hipError_t launch_cipher_variant(int grid_mult, uint64_t max_blocks, const tdes_msg *msgs,
                                 uint32_t n_msgs, const uint32_t *sched, uint32_t n_sched,
                                 const uint8_t *in, uint8_t *out, const uint64_t *ws,
                                 hipStream_t stream) {
    uint64_t blocks = (uint64_t)resident_blocks<K, W>() * (uint64_t)grid_mult;
    if (max_blocks != 0 && max_blocks < blocks) blocks = max_blocks;
    hipLaunchKernelGGL((batch_bitslice_kernel<K, W>), dim3((unsigned)blocks), dim3(kThreads), 0,
                       stream, msgs, n_msgs, sched, n_sched, in, out, ws);
    return hipGetLastError();
}

// The batched cipher in the current device's configuration.
hipError_t launch_cipher(const tdes_msg *msgs, size_t n_msgs, const uint32_t *sched,
                         size_t n_sched, const uint8_t *in, uint8_t *out, const uint64_t *ws,
                         uint64_t max_blocks, hipStream_t stream) {
    BatchConfig c;
    const hipError_t e = batch_config_current(&c);
    if (e != hipSuccess) return e;
#define TDES_LAUNCH_IF(K, W)                                                                   \
    if (c.kmax == K && c.waves == W)                                                           \
        return launch_cipher_variant<K, W>(c.grid_mult, max_blocks, msgs, (uint32_t)n_msgs,     \
                                           sched, (uint32_t)n_sched, in, out, ws, stream);
    TDES_BATCH_VARIANTS(TDES_LAUNCH_IF)
#undef TDES_LAUNCH_IF
    return hipErrorInvalidValue;
}

}  // namespace

bool batch_config_valid(const BatchConfig &c) {
    if (c.grid_mult < 1 || c.grid_mult > kMaxGridMult) return false;
#define TDES_VALID_IF(K, W) \
    if (c.kmax == K && c.waves == W) return true;
    TDES_BATCH_VARIANTS(TDES_VALID_IF)
#undef TDES_VALID_IF
    return false;
}

BatchConfig batch_config_default() { return kDefaultConfig; }

int batch_config_list(BatchConfig *out, int cap) {
    int n = 0;
#define TDES_LIST(K, W)                                                                   \
    for (int m = 1; m <= kMaxGridMult; m++, n++)                                          \
        if (n < cap) out[n] = BatchConfig{K, W, m};
    TDES_BATCH_VARIANTS(TDES_LIST)
#undef TDES_LIST
    return n;
}

hipError_t launch_expand(const uint8_t *keys24, size_t n, uint32_t *schedules, hipStream_t stream) {
    const size_t blocks = (n + kExpandWaves - 1) / kExpandWaves;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(expand_kernel, dim3((unsigned)blocks), dim3(kExpandWaves * kWave), 0, stream,
                       keys24, n, schedules);
    return hipGetLastError();
}

hipError_t launch_batch_prefixed(const tdes_msg *msgs, size_t n_msgs, const uint32_t *schedules,
                                 size_t n_schedules, const uint8_t *in, uint8_t *out,
                                 const uint64_t *ws, uint64_t total_slices, hipStream_t stream) {
    // a workgroup's waves take kWave consecutive slices each per step
    const uint64_t per_block = (uint64_t)kWave * kWavesPerBlock;
    const uint64_t need = total_slices == 0 ? 1 : (total_slices + per_block - 1) / per_block;
    return launch_cipher(msgs, n_msgs, schedules, n_schedules, in, out, ws, need, stream);
}

hipError_t batch_autotune(const tdes_msg *msgs, size_t n_msgs, const uint32_t *schedules,
                          size_t n_schedules, const uint8_t *in, uint64_t in_bytes,
                          const TuneLane *lanes, int n_lanes, uint64_t out_bytes, int reps,
                          BatchConfig *best_out, float *best_us) {
    if (n_lanes < 1 || n_lanes > kMaxTuneLanes) return hipErrorInvalidValue;
    BatchConfig keep;
    hipError_t e = batch_config_current(&keep);
    if (e != hipSuccess) return e;
    BatchConfig cands[64];
    const int n_cands = batch_config_list(cands, 64);
    // a: start, on lane 0's stream, which the other lanes wait for; end[i]:
    // lane i's last batch, which lane 0 waits for before b
    hipEvent_t a = nullptr, b = nullptr, end[kMaxTuneLanes] = {};
    e = hipEventCreateWithFlags(&a, hipEventDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b, hipEventDefault);
    for (int i = 1; i < n_lanes && e == hipSuccess; i++)
        e = hipEventCreateWithFlags(&end[i], hipEventDisableTiming);
    float best_ms = 0;
    BatchConfig best = keep;
    auto run = [&](const TuneLane &l) {
        return launch_batch(msgs, n_msgs, schedules, n_schedules, in, in_bytes, l.out, out_bytes,
                            l.ws, nullptr, l.stream);
    };
    const hipStream_t s0 = lanes[0].stream;
    for (int i = 0; i < n_cands && e == hipSuccess; i++) {
        e = batch_config_set(cands[i]);
        for (int l = 0; l < n_lanes && e == hipSuccess; l++) e = run(lanes[l]);  // warm
        for (int l = 0; l < n_lanes && e == hipSuccess; l++) e = hipStreamSynchronize(lanes[l].stream);
        if (e == hipSuccess) e = hipEventRecord(a, s0);
        for (int l = 1; l < n_lanes && e == hipSuccess; l++) e = hipStreamWaitEvent(lanes[l].stream, a, 0);
        // back-to-back batches, taking the lanes in turn
        for (int r = 0; r < reps * n_lanes && e == hipSuccess; r++) e = run(lanes[r % n_lanes]);
        for (int l = 1; l < n_lanes && e == hipSuccess; l++) {
            e = hipEventRecord(end[l], lanes[l].stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(s0, end[l], 0);
        }
        if (e == hipSuccess) e = hipEventRecord(b, s0);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && (i == 0 || ms < best_ms)) {
            best_ms = ms;
            best = cands[i];
        }
    }
    (void)batch_config_set(e == hipSuccess ? best : keep);
    if (a != nullptr) (void)hipEventDestroy(a);
    if (b != nullptr) (void)hipEventDestroy(b);
    for (int l = 1; l < n_lanes; l++)
        if (end[l] != nullptr) (void)hipEventDestroy(end[l]);
    if (e == hipSuccess) {
        *best_out = best;
        *best_us = best_ms * 1e3f / (float)(reps * n_lanes);
    }
    return e;
}

size_t batch_workspace_bytes(size_t n_msgs) {
    const size_t tiles = (n_msgs + kTile - 1) / kTile;
    return (kWsHeader + n_msgs + 1 + 2 * tiles) * sizeof(uint64_t);
}

// The workspace of the no-allocation entry point: a fixed array in device
// memory (each device holds its own copy), sized for TDES_BATCH_NOALLOC_MAX_MSGS
// messages.  In host code its name is not a device address; the address is
// looked up once per device (with that device current) and kept.
static_assert(TDES_BATCH_NOALLOC_MAX_MSGS <= TDES_BATCH_MAX_MSGS, "no-alloc limit");
constexpr size_t kNoAllocWords = kWsHeader + (size_t)TDES_BATCH_NOALLOC_MAX_MSGS + 1 +
                                 2 * (((size_t)TDES_BATCH_NOALLOC_MAX_MSGS + kTile - 1) / kTile);
static __device__ __align__(256) uint64_t scratch[kNoAllocWords];

hipError_t noalloc_workspace(uint64_t **ws, size_t *ws_bytes) {
    static std::atomic<uint64_t *> addr[kMaxDevices];
    static std::mutex mu;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    uint64_t *p = addr[dev].load();
    if (p == nullptr) {
        std::lock_guard<std::mutex> g(mu);
        p = addr[dev].load();
        if (p == nullptr) {
            void *sym = nullptr;
            e = hipGetSymbolAddress(&sym, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            if (sym == nullptr) return hipErrorInvalidSymbol;
            p = static_cast<uint64_t *>(sym);
            addr[dev].store(p);
        }
    }
    *ws = p;
    *ws_bytes = kNoAllocWords * sizeof(uint64_t);
    return hipSuccess;
}

hipError_t launch_batch(const tdes_msg *msgs, size_t n_msgs, const uint32_t *schedules,
                        size_t n_schedules, const uint8_t *in, uint64_t in_bytes, uint8_t *out,
                        uint64_t out_bytes, uint64_t *ws, uint64_t *skipped_out,
                        hipStream_t stream) {
    const size_t T = (n_msgs + kTile - 1) / kTile;  // n_msgs >= 1
    if (T > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_tile_scan_kernel, dim3((unsigned)T), dim3(kScanThreads), 0, stream,
                       msgs, n_msgs, n_schedules, BatchBounds{in_bytes, out_bytes}, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (T <= kFusedTiles) {
        hipLaunchKernelGGL(batch_tile_finish_kernel, dim3((unsigned)T), dim3(kScanThreads), 0,
                           stream, n_msgs, ws, skipped_out);
    } else {
        hipLaunchKernelGGL(batch_tile_offsets_kernel, dim3(1), dim3(kScanThreads), 0, stream,
                           n_msgs, ws, skipped_out);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(batch_tile_add_kernel, dim3((unsigned)T), dim3(kScanThreads), 0, stream,
                           n_msgs, ws);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_cipher(msgs, n_msgs, schedules, n_schedules, in, out, ws, 0, stream);
}

}  // namespace tdes
