// Declarations shared by the host side of the library (not part of the ABI).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>

#include <hip/hip_runtime_api.h>

#include "keysched_core.h"
#include "tdes.h"

namespace tdes {

// The 48 round keys one 3DES pass applies, in application order
// (Sec. III-B equations; decryption of one DES stage = its keys reversed).
struct RoundSequence {
    uint64_t rk[48];  // 48-bit round keys, bit 1 = bit 47
};

// Kernel argument for the bitsliced kernel: the 100 key-mask words of one
// direction (layout in keysched_core.h); the kernel expands the bits to
// 0 / ~0 words in LDS.
struct BitsliceKeys {
    uint32_t w[100];
};

// Per-launch arguments of the bitsliced kernel's modes (ECB ignores them).
enum : int { kModeEcb = 0, kModeCtr = 1, kModeCbcDec = 2 };
struct ModeArgs {
    uint64_t ctr;       // CTR: counter of the buffer's first block (big-endian value)
    uint32_t iv0, iv1;  // CBC: the IV's bytes 0-3 and 4-7, little-endian words
};

// Kernel argument for the one-thread-per-bit comparison kernel: the 16
// round keys of one DES pass in application order, one byte (0 or 1) per
// key bit, round i at 48 i (bit 1 first).
struct ReplicaKeyBits {
    uint8_t k[16 * 48];
};

// Kernel argument for the table kernel: per round, the key chunks XORed into
// the right half where the S-box windows sit (see spbox.hip): odd chunks,
// even chunks, chunks 0 and 6 and chunk 7 for the half rotated left by 12.
struct SpboxKeys {
    uint32_t w[48][4];
};

// Device-resident key material of one schedule (tdes_schedule_upload,
// tdes_schedule_expand): the 100 mask words (keysched_core.h) of
// encryption, then those of decryption.
constexpr int kDeviceScheduleWords = 200;
static_assert(kDeviceScheduleWords * 4 == TDES_DEVICE_SCHEDULE_BYTES, "schedule size");

// Record msg as the calling thread's last error (tdes_last_error) and
// return st.
tdes_status set_last_error(tdes_status st, const char *msg);

void device_schedule_words(const tdes_schedule &ks, uint32_t out[kDeviceScheduleWords]);
void round_sequence(const tdes_schedule &ks, int dir, RoundSequence *seq);
void bitslice_keys(const tdes_schedule &ks, int dir, BitsliceKeys *out);
void spbox_keys(const RoundSequence &seq, SpboxKeys *out);

// Launchers: enqueue on `stream`; return the HIP launch status.
hipError_t launch_bitslice(const BitsliceKeys &k, const uint8_t *in, uint8_t *out,
                           size_t nbytes, hipStream_t stream);
// CTR mode: out = in XOR E(counter blocks ctr, ctr + 1, ...), k = encryption keys.
hipError_t launch_bitslice_ctr(const BitsliceKeys &k, uint64_t ctr, const uint8_t *in,
                               uint8_t *out, size_t nbytes, hipStream_t stream);
// CBC decryption: out block i = D(in block i) XOR in block i - 1 (the IV for
// i = 0), k = decryption keys; in and out must not overlap.
hipError_t launch_bitslice_cbc_dec(const BitsliceKeys &k, uint32_t iv0, uint32_t iv1,
                                   const uint8_t *in, uint8_t *out, size_t nbytes,
                                   hipStream_t stream);
size_t batch_workspace_bytes(size_t n_msgs);

// Configuration of the batched cipher: the compiled variant (kmax messages
// per mask-table group, waves per SIMD) and the grid in multiples of the
// workgroups that fit at once.
struct BatchConfig {
    int kmax, waves, grid_mult;
};
bool batch_config_valid(const BatchConfig &c);  // a compiled variant, grid_mult 1..4
BatchConfig batch_config_default();
// Every valid configuration (variants x multipliers), up to cap; returns
// their number.
int batch_config_list(BatchConfig *out, int cap);
// The configuration batched launches use on the current device: set by
// batch_config_set, else on first use the tuning cache's entry for this
// device kind, else the default.
hipError_t batch_config_current(BatchConfig *out);
hipError_t batch_config_set(const BatchConfig &c);
// Write c as this device kind's entry of the tuning cache (true if written,
// or if the cache is switched off).
bool batch_config_persist(const BatchConfig &c, double us_per_batch);
// The tuning cache file: $TDES_TUNE_CACHE ("" = none), else
// $XDG_CACHE_HOME/tdes/batch_tune.json, else ~/.cache/tdes/batch_tune.json.
std::string tune_cache_path();
// Entry of (device, cus) in the cache file at path: 1 found (and valid),
// 0 none, -1 bad arguments.
int cache_load(const char *path, const char *device, long cus, BatchConfig *out);
bool cache_save(const char *path, const char *device, long cus, const BatchConfig &c,
                double us_per_batch);
hipError_t launch_expand(const uint8_t *keys24, size_t n, uint32_t *schedules, hipStream_t stream);
// The batched cipher alone, for a workspace whose first-slice table the
// caller filled already ([0] total slices, [1] 0, [2 + i] first slice of
// message i, [2 + n] total; a message has ceil(nbytes / 256) slices).  The
// grid is no larger than total_slices needs.
hipError_t launch_batch_prefixed(const tdes_msg *msgs, size_t n_msgs, const uint32_t *schedules,
                                 size_t n_schedules, const uint8_t *in, uint8_t *out,
                                 const uint64_t *ws, uint64_t total_slices, hipStream_t stream);
// Descriptor scan (validation against the buffer sizes, first-slice table in
// ws, skipped count in ws[1] and, if skipped_out is not NULL, there too),
// then the batched cipher.
hipError_t launch_batch(const tdes_msg *msgs, size_t n_msgs, const uint32_t *schedules,
                        size_t n_schedules, const uint8_t *in, uint64_t in_bytes, uint8_t *out,
                        uint64_t out_bytes, uint64_t *ws, uint64_t *skipped_out,
                        hipStream_t stream);
// The fixed device workspace of the no-allocation batched call on the
// current device (its address, looked up on the first call on that device,
// and its size in bytes).
hipError_t noalloc_workspace(uint64_t **ws, size_t *ws_bytes);
// One lane of the autotuner: an output buffer, a workspace and a stream of
// its own.
struct TuneLane {
    uint8_t *out;
    uint64_t *ws;
    hipStream_t stream;
};
constexpr int kMaxTuneLanes = 8;
// Times the batch (scan + cipher) in every configuration: after one warm run
// per lane, reps x n_lanes back-to-back submits taking the lanes in turn
// (with one lane, on one stream; with several, batches overlap across the
// lanes' streams).  Keeps the fastest for later batched launches on the
// current device and returns it with its time per batch (us).  Synchronous.
hipError_t batch_autotune(const tdes_msg *msgs, size_t n_msgs, const uint32_t *schedules,
                          size_t n_schedules, const uint8_t *in, uint64_t in_bytes,
                          const TuneLane *lanes, int n_lanes, uint64_t out_bytes, int reps,
                          BatchConfig *best, float *best_us);
// Bytes the table kernel covers with one block per lane in one wave of
// resident workgroups on the current device (4 MiB on 256 CUs).  Up to 1.5
// times this size it has the lower latency: its lanes each run one or two
// blocks through the rounds, while a bitsliced lane runs 32 (one launch of
// either kernel measured 8-29 us against 33-35 us); above it the bitsliced
// kernel's throughput wins.
size_t spbox_one_pass_bytes();

// tdes_ecb_crypt's TDES_KERNEL_AUTO: the table kernel up to one and a half
// times spbox_one_pass_bytes(), the bitsliced kernel above (auto_kernel says which,
// as a tdes_kernel value).
int auto_kernel(size_t nbytes);
hipError_t launch_ecb_auto(const tdes_schedule &ks, int dir, const uint8_t *in, uint8_t *out,
                           size_t nbytes, hipStream_t stream);

hipError_t launch_spbox(const SpboxKeys &k, const uint8_t *in, uint8_t *out, size_t nbytes,
                        hipStream_t stream);

// The table kernel over several messages in one launch, each with its own
// keys (the request server's small batches).  Message i's blocks go to
// workgroups first_wg .. first_wg + ceil(nblocks / per) - 1, `per` blocks
// each; first_wg of message 0 is 0 and the values do not decrease.
struct SpboxMsg {
    const uint8_t *in;
    uint8_t *out;
    uint64_t nblocks;
    uint32_t first_wg;
    uint32_t pad;
};
constexpr uint32_t kSpboxMultiMax = 64;  // messages per launch
// Working lanes per workgroup for messages of these block counts: the fewest
// of 64, 128, .. 1,024 whose workgroups fit the CUs once (1,024 if none).
uint32_t spbox_multi_lanes(const uint64_t *nblocks, size_t n);
// d_msgs: n device descriptors (1 <= n <= kSpboxMultiMax); d_keys: n
// SpboxKeys in device memory, 16-byte aligned; n_wg: the workgroups the
// descriptors cover (first_wg + ceil(nblocks / per) of the last message).
hipError_t launch_spbox_multi(const SpboxMsg *d_msgs, uint32_t n, const SpboxKeys *d_keys,
                              uint32_t per, uint32_t n_wg, hipStream_t stream);

// One DES pass of the one-thread-per-bit comparison kernel (in may equal out).
hipError_t launch_replica_pass(const ReplicaKeyBits &k, const uint8_t *in, uint8_t *out,
                               size_t nbytes, hipStream_t stream);

// Host-resident pipeline behind tdes_ecb_host (arguments already checked):
// chunks of `chunk` bytes through n_slots device slots at d_work; returns
// once every chunk is back in h_out, or the first HIP error.
hipError_t run_host_pipeline(const BitsliceKeys &k, const uint8_t *h_in, uint8_t *h_out,
                             size_t nbytes, uint8_t *d_work, size_t n_slots, size_t chunk);
// Device address *d of the host range [h, h + n), n > 0: an error unless
// the whole range lies in one pinned, device-mapped host allocation.
hipError_t mapped_range(const void *h, size_t n, uint8_t **d);
// The kernel run in place on device-mapped host memory (device addresses
// from mapped_range); returns once it has finished, or the first HIP error.
hipError_t run_host_direct(const BitsliceKeys &k, const uint8_t *d_in, uint8_t *d_out,
                           size_t nbytes);

}  // namespace tdes
