/*
 * tdes.h - Triple-DES (EDE) over independent 64-bit blocks on one AMD
 * Instinct MI355X (gfx950), C ABI.
 *
 * Method: the DES key schedule (Sec. III-A of the paper: PC-1, cumulative
 * left rotations by the shift table, PC-2, 16 round keys per base key),
 * DES block encryption and decryption (Sec. III-B: IP, 16 Feistel rounds of
 * expansion, key mixing, S-boxes and the straight permutation, R16 || L16,
 * FP; decryption uses the round keys in reverse), composed as 3DES-EDE
 *     C = E_K3(D_K2(E_K1(P))),   P = D_K1(E_K2(D_K3(C)))   (Sec. III-B)
 * and applied to every 8-byte block independently (ECB, Sec. V).
 *
 * Conventions
 *   - DES bit 1 is the most significant bit of byte 0 of a key or block.
 *   - A key bundle is 24 bytes K1 || K2 || K3; 2-key 3DES is K1 || K2 || K1.
 *     Parity bits (bit 8 of every key byte) are ignored, never checked.
 *   - Lengths are in bytes and must be a multiple of 8; no padding is added.
 *   - Device pointers are plain HIP device addresses (for example the
 *     data_ptr() of a torch tensor); the caller owns every buffer.  The
 *     library allocates no memory on the encryption path (tdes_ecb_host
 *     creates its streams once per device).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device calls
 *     only enqueue work and return; results are valid once the stream has
 *     completed the work.  tdes_ecb_host, which takes host buffers, is
 *     synchronous instead.
 *   - Argument errors are reported synchronously, before any device work is
 *     enqueued; a failed launch returns TDES_ERR_DEVICE.  tdes_last_error()
 *     gives a message for the last failure on the calling thread.  No C++
 *     exception crosses this interface.
 */
#ifndef TDES_H
#define TDES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDES_ABI_VERSION 3

typedef enum {
    TDES_OK = 0,
    TDES_ERR_ARG = -1,        /* NULL pointer or bad enum value            */
    TDES_ERR_LENGTH = -2,     /* byte count not a multiple of 8            */
    TDES_ERR_ALIGN = -3,      /* device pointer not 8-byte aligned         */
    TDES_ERR_OVERLAP = -4,    /* input and output overlap but differ       */
    TDES_ERR_NOMEM = -5,      /* reserved: the library does not allocate   */
    TDES_ERR_DEVICE = -6      /* HIP reported an error; see last_error     */
} tdes_status;

typedef enum { TDES_ENCRYPT = 0, TDES_DECRYPT = 1 } tdes_dir;

/* Kernel selection for tdes_ecb_crypt. */
typedef enum {
    TDES_KERNEL_AUTO = 0,     /* the library's choice: the table kernel up
                                 to 1.5 times the bytes one wave of its
                                 resident workgroups covers at one block per
                                 lane (6 MiB on 256 CUs; lower latency), the
                                 bitsliced kernel above (higher throughput) */
    TDES_KERNEL_BITSLICE = 1, /* 32 blocks per lane as bit planes; S-boxes
                                 as gate networks, E/P/IP/FP as renaming   */
    TDES_KERNEL_SPBOX = 2     /* one block per lane; S-box+P tables in LDS */
} tdes_kernel;

/* The kernel TDES_KERNEL_AUTO runs for nbytes on the current device:
 * TDES_KERNEL_SPBOX up to 1.5 times the table kernel's one-pass size
 * (resident workgroups x 1,024 lanes x 8 bytes: 6 MiB on 256 CUs),
 * TDES_KERNEL_BITSLICE above.  Returns a negative tdes_status (TDES_ERR_DEVICE) without a
 * device. */
int tdes_ecb_auto_kernel(size_t nbytes);

/* Round keys of a key bundle, Sec. III-A.  k[b][i] is round key i+1 (of 16)
 * of base key K(b+1), 48 bits, with round-key bit 1 as bit 47 of the value.
 * A plain value type: copy it, keep it on the host. */
typedef struct {
    uint64_t k[3][16];
} tdes_schedule;

/* Key generation (Sec. III-A) for the 24-byte bundle key24 (host memory).
 * Synchronous, host only.  Errors: TDES_ERR_ARG on NULL. */
tdes_status tdes_key_schedule(const uint8_t key24[24], tdes_schedule *out);

/* 3DES-EDE ECB encryption of nbytes bytes at device address d_in into
 * d_out (Sec. III-B; ECB, Sec. V).  d_in == d_out (in place) is allowed;
 * any other overlap is TDES_ERR_OVERLAP.  nbytes == 0 is a no-op.
 * Errors: TDES_ERR_ARG (NULL ks or buffers with nbytes > 0),
 * TDES_ERR_LENGTH (nbytes % 8), TDES_ERR_ALIGN (pointer % 8),
 * TDES_ERR_OVERLAP, TDES_ERR_DEVICE (launch failure). */
tdes_status tdes_ecb_encrypt(const tdes_schedule *ks, const void *d_in, void *d_out,
                             size_t nbytes, void *stream);

/* 3DES-EDE ECB decryption; same arguments and errors as tdes_ecb_encrypt. */
tdes_status tdes_ecb_decrypt(const tdes_schedule *ks, const void *d_in, void *d_out,
                             size_t nbytes, void *stream);

/* Encryption or decryption (dir) with an explicit kernel choice; same
 * arguments and errors as tdes_ecb_encrypt, plus TDES_ERR_ARG for a bad
 * dir or kernel value. */
tdes_status tdes_ecb_crypt(const tdes_schedule *ks, int dir, int kernel, const void *d_in,
                           void *d_out, size_t nbytes, void *stream);

/* 3DES-EDE in counter mode over device memory (CTR, NIST SP 800-38A
 * Sec. 6.5; the paper itself uses ECB only, Sec. V).  Output block i is
 * input block i XOR E(T_i), where E is the 3DES-EDE encryption of
 * Sec. III-B with bundle ks.  The counter block T_i is (IV + i) mod 2^64,
 * the whole 64-bit block read as a big-endian integer; iv points to its
 * 8 bytes (host memory).  Encryption and decryption are the same
 * operation.  The counter blocks are made in the kernel, so only the data
 * is read.  Buffers, stream and errors as for tdes_ecb_encrypt, plus
 * TDES_ERR_ARG for a NULL iv. */
tdes_status tdes_ctr_crypt(const tdes_schedule *ks, const uint8_t iv[8], const void *d_in,
                           void *d_out, size_t nbytes, void *stream);

/* 3DES-EDE CBC decryption over device memory (NIST SP 800-38A Sec. 6.2;
 * the paper itself uses ECB only, Sec. V): output block i is
 * D(input block i) XOR input block i - 1, with the IV (8 bytes, host
 * memory) in place of input block -1.  D is the 3DES-EDE decryption of
 * Sec. III-B with bundle ks.  Every block is independent of the other
 * blocks' results, so it runs at full width; CBC encryption is serial
 * within a message and is not offered.  The ciphertext blocks before each
 * block are re-read from d_in, so d_in and d_out must not overlap at all
 * (in place is TDES_ERR_OVERLAP).  Otherwise buffers, stream and errors as
 * for tdes_ecb_decrypt, plus TDES_ERR_ARG for a NULL iv. */
tdes_status tdes_cbc_decrypt(const tdes_schedule *ks, const uint8_t iv[8], const void *d_in,
                             void *d_out, size_t nbytes, void *stream);

/* The paper's own GPU design (Sec. IV-B, IV-C), for comparison only: one
 * 64-thread workgroup per block, one thread per bit, bits one per byte in
 * LDS, tables read at run time, a barrier between steps, and three launches
 * (one per DES pass; decryption passes take their round keys reversed, as
 * the paper does on the host).  Same result as tdes_ecb_crypt; far slower.
 * Buffers, stream and errors as for tdes_ecb_crypt (no kernel argument). */
tdes_status tdes_ecb_paper_design(const tdes_schedule *ks, int dir, const void *d_in, void *d_out,
                                  size_t nbytes, void *stream);

/* ---- Batched form: many messages, each with its own key and direction --- */

/* Bytes of device-resident key material per schedule (both directions). */
#define TDES_DEVICE_SCHEDULE_BYTES 800

/* One message of a batch (device memory, 32 bytes).  The message is nbytes
 * bytes (a multiple of 8) at byte offset in_off of the batch's input base
 * and its result goes to out_off of the output base (both multiples of 8;
 * in_off == out_off on the same base is in place).  It is encrypted or
 * decrypted (dir) with schedule sched_idx of the batch's device schedules.
 * Messages must not overlap each other's outputs. */
typedef struct {
    uint64_t in_off;
    uint64_t out_off;
    uint64_t nbytes;
    uint32_t sched_idx;
    uint32_t dir;
} tdes_msg;

/* Write the device-resident key material of n schedules (host memory h) to
 * d_dst (device, n * TDES_DEVICE_SCHEDULE_BYTES bytes, 16-byte aligned,
 * owned by the caller).  The copy is enqueued on `stream` and waited for:
 * h may be reused on return.  Errors: TDES_ERR_ARG, TDES_ERR_ALIGN,
 * TDES_ERR_DEVICE. */
tdes_status tdes_schedule_upload(const tdes_schedule *h, size_t n, void *d_dst, void *stream);

/* The key generation of Sec. III-A on the device, for many bundles at once
 * (the role of the paper's key-generation kernel, Sec. IV-A, applied to a
 * whole batch): n key bundles of 24 bytes (K1 || K2 || K3) at d_keys24
 * (device) become n device-resident schedules at d_schedules (device,
 * n * TDES_DEVICE_SCHEDULE_BYTES bytes, 16-byte aligned), the same bytes
 * tdes_schedule_upload writes.  Asynchronous on `stream`.  Errors:
 * TDES_ERR_ARG, TDES_ERR_ALIGN, TDES_ERR_DEVICE. */
tdes_status tdes_schedule_expand(const void *d_keys24, size_t n, void *d_schedules, void *stream);

/* Most messages and schedules one batched call takes (TDES_ERR_ARG beyond). */
#define TDES_BATCH_MAX_MSGS (1u << 31)
#define TDES_BATCH_MAX_SCHEDULES (1u << 22)

/* Device workspace bytes tdes_batch_submit needs for n_msgs messages. */
size_t tdes_batch_workspace_bytes(size_t n_msgs);

/* 3DES-EDE ECB over a batch of messages in one pass (the batched form of
 * tdes_ecb_crypt: per-message keys and directions, Sec. III-B; ECB, Sec. V).
 * d_msgs: n_msgs descriptors in device memory; d_schedules: n_schedules
 * entries written by tdes_schedule_upload or tdes_schedule_expand;
 * d_in_base / d_out_base: device buffers of in_bytes / out_bytes bytes that
 * the message offsets refer to (8-byte aligned); d_workspace:
 * tdes_batch_workspace_bytes(n_msgs) bytes of device memory (8-byte aligned),
 * overwritten.  Asynchronous on `stream`.  Message fields are checked on the
 * device: a message whose length or offsets are not multiples of 8, whose
 * input range [in_off, in_off + nbytes) exceeds in_bytes or output range
 * [out_off, out_off + nbytes) exceeds out_bytes, or whose schedule index or
 * direction is out of range is skipped (neither read nor written), and the
 * number skipped is left in the second 64-bit word of the workspace.
 * Messages whose outputs overlap each other are not detected; their bytes
 * are then unspecified.  Errors (synchronous): TDES_ERR_ARG (NULL pointers
 * with n_msgs > 0, workspace too small, n_msgs > TDES_BATCH_MAX_MSGS,
 * n_schedules 0 or > TDES_BATCH_MAX_SCHEDULES), TDES_ERR_ALIGN,
 * TDES_ERR_DEVICE. */
tdes_status tdes_batch_submit(const tdes_msg *d_msgs, size_t n_msgs, const void *d_schedules,
                              size_t n_schedules, const void *d_in_base, size_t in_bytes,
                              void *d_out_base, size_t out_bytes, void *d_workspace,
                              size_t workspace_bytes, void *stream);

/* Most messages one tdes_batch_submit_noalloc call takes. */
#define TDES_BATCH_NOALLOC_MAX_MSGS (1u << 20)

/* tdes_batch_submit without a caller workspace and without any allocation,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * descriptor scan's table lives in a fixed array in the library's device
 * memory (8 MiB + 16 KiB + 24 bytes: room for TDES_BATCH_NOALLOC_MAX_MSGS messages),
 * one per device, held until the process ends; its address is looked up on
 * the first call on each device.  Nothing in it must start at zero: the
 * scan rewrites what the cipher reads on every call.  Every call on a device
 * shares that device's array, so calls whose work overlaps in time on one
 * device (other streams, other threads) race and their results are
 * unspecified: serialise them, for example on one stream.  Arguments, checks
 * and results as for tdes_batch_submit, except: d_skipped (device memory,
 * 8-byte aligned, or NULL) receives the number of skipped messages, and
 * n_msgs > TDES_BATCH_NOALLOC_MAX_MSGS is TDES_ERR_ARG.  Calls no hipMalloc
 * or hipFree. */
tdes_status tdes_batch_submit_noalloc(const tdes_msg *d_msgs, size_t n_msgs,
                                      const void *d_schedules, size_t n_schedules,
                                      const void *d_in_base, size_t in_bytes, void *d_out_base,
                                      size_t out_bytes, uint64_t *d_skipped, void *stream);

/* ---- Host-resident form: data in host memory ----------------------------- */

/* Most slots (device staging buffers, one stream each) tdes_ecb_host uses. */
#define TDES_HOST_MAX_SLOTS 8

/* 3DES-EDE ECB (Sec. III-B; ECB, Sec. V) of nbytes bytes of HOST memory
 * h_in into host memory h_out, through the device.  The paper's input
 * starts on the host (Sec. IV-C) and its GPU times leave the transfers out
 * (Sec. V); this call includes them.  Two modes:
 *
 *   - Direct (d_work == NULL): h_in and h_out must be pinned host memory
 *     (hipHostMalloc), which is mapped into the device's address space.  The
 *     bitsliced kernel reads and writes them there, over PCIe in both
 *     directions at once; nothing is staged.  chunk_bytes and work_bytes
 *     are ignored.  Each range must lie within one pinned allocation
 *     (checked: TDES_ERR_ARG otherwise).
 *   - Staged (d_work != NULL): any host memory.  The range is cut into
 *     chunks of chunk_bytes (the last one shorter).  Chunk i goes to slot
 *     i % n_slots of the device workspace d_work (n_slots =
 *     min(work_bytes / chunk_bytes, TDES_HOST_MAX_SLOTS)).  There it is
 *     copied in, encrypted or decrypted in place by the bitsliced kernel,
 *     and copied out, in order on that slot's stream.  The slots' streams
 *     run side by side, so copies to the device, kernels and copies back of
 *     different chunks overlap.  The copies run asynchronously only if the
 *     host buffers are pinned; pageable memory gives the same result, more
 *     slowly.  d_work is caller-owned device memory, 256-byte aligned, at
 *     least chunk_bytes long, not in use by pending device work.  A
 *     chunk_bytes that is a multiple of 16 KiB keeps every slot 16-byte
 *     aligned, the kernel's fast path.
 *
 * Streams: both modes run on streams that belong to the library.  There is
 * one set per device, at default priority, created at the first call on
 * that device and kept until the process ends.
 *
 * Buffers: h_in == h_out (in place) is allowed; any other overlap is
 * TDES_ERR_OVERLAP.  The caller owns every buffer.
 *
 * Synchronous, unlike the device calls: it returns once h_out holds the
 * result or an error occurred.  Calls from several threads are serialised.
 * nbytes == 0 is a no-op.
 *
 * Errors, all reported before any device work:
 *   - TDES_ERR_ARG: NULL ks or buffers with nbytes > 0, or a bad dir.
 *     Direct mode: unmapped buffers.  Staged mode: chunk_bytes 0, or
 *     work_bytes < chunk_bytes;
 *   - TDES_ERR_LENGTH: nbytes, or (staged) chunk_bytes, not a multiple
 *     of 8;
 *   - TDES_ERR_ALIGN: h_in or h_out not 8-byte aligned, or (staged) d_work
 *     not 256-byte aligned;
 *   - TDES_ERR_OVERLAP: see above.
 * TDES_ERR_DEVICE is returned if a HIP call fails.  The contents of h_out
 * are then unspecified. */
tdes_status tdes_ecb_host(const tdes_schedule *ks, int dir, const void *h_in, void *h_out,
                          size_t nbytes, void *d_work, size_t work_bytes, size_t chunk_bytes);

/* Configuration of the batched kernel: which compiled variant runs and on
 * how large a grid.  None of it changes results, only speed. */
typedef struct {
    uint32_t kmax;      /* messages per wave pass whose key masks share one LDS
                           table (4, 8 or 16; a wave over more messages takes
                           one pass per group)                              */
    uint32_t waves;     /* waves per SIMD the variant's register budget is
                           set for.  Compiled: {4, 8} x {3, 4, 5} and
                           {16, 3}                                          */
    uint32_t grid_mult; /* grid = grid_mult x the workgroups that fit at
                           once (1..4)                                      */
    uint32_t saved;     /* output of tdes_batch_autotune: 1 if the result was
                           written to the tuning cache; ignored on input    */
} tdes_batch_config;

/* The configuration batched calls use on the current device.  Until it is
 * set (tdes_batch_set_config, tdes_batch_autotune) it is, from the first
 * batched call on, the tuning cache's entry for this kind of device (same
 * architecture name and compute-unit count), else the default
 * {8, 4, 2}.  The tuning cache is the JSON file named by TDES_TUNE_CACHE
 * (empty: no cache), else $XDG_CACHE_HOME/tdes/batch_tune.json, else
 * ~/.cache/tdes/batch_tune.json.  Errors: TDES_ERR_ARG (NULL),
 * TDES_ERR_DEVICE (no device). */
tdes_status tdes_batch_get_config(tdes_batch_config *out);

/* Set the configuration for later batched calls on the current device (the
 * request server's batches included).  Errors: TDES_ERR_ARG (NULL, or not
 * a compiled variant, or grid_mult outside 1..4), TDES_ERR_DEVICE. */
tdes_status tdes_batch_set_config(const tdes_batch_config *cfg);

/* Autotuner for the batched form: runs this batch (arguments and checks as
 * for tdes_batch_submit) in every configuration (each compiled variant at
 * grids of 1, 2, 3 and 4 times the workgroups that fit at once), reps
 * (>= 1) times each after one warm run, timed with HIP events on
 * `stream`.  The fastest is kept for every later batched call on the
 * current device (the request server's batches included), written to the
 * tuning cache under this device kind (best->saved says whether it was),
 * and returned in *best.  Synchronous.  Every trial reads the input and
 * writes the output, so the input range [d_in_base, d_in_base + in_bytes)
 * must not overlap the output range (TDES_ERR_OVERLAP otherwise, in-place
 * batches included): each trial then writes the same result.  Batched
 * calls from other threads on the same device while it runs use the
 * configuration under trial (same results, other speed).  Errors: those of
 * tdes_batch_submit, TDES_ERR_OVERLAP, and TDES_ERR_ARG for reps < 1 or a
 * NULL best. */
tdes_status tdes_batch_autotune(const tdes_msg *d_msgs, size_t n_msgs, const void *d_schedules,
                                size_t n_schedules, const void *d_in_base, size_t in_bytes,
                                void *d_out_base, size_t out_bytes, void *d_workspace,
                                size_t workspace_bytes, void *stream, int reps,
                                tdes_batch_config *best);

/* The autotuner for a stream of batches, run the way a server runs them:
 * each configuration is timed over reps x n_streams
 * back-to-back submits of this batch taking the n_streams lanes in turn,
 * lane i writing d_out_bases[i] with workspace d_workspaces[i] on
 * streams[i], so that batches on different streams overlap (one batch's
 * last waves beside the next one's first).  The fastest configuration per
 * batch is kept, saved and returned as by tdes_batch_autotune, which is this
 * call with one lane.  Arrays of n_streams (1..8) host pointers; each
 * output and workspace must not overlap another lane's, nor an output the
 * input (TDES_ERR_OVERLAP); the other checks are tdes_batch_submit's, per
 * lane.  Synchronous.  Errors: those of tdes_batch_autotune, and
 * TDES_ERR_ARG for NULL arrays or n_streams outside 1..8. */
tdes_status tdes_batch_autotune_streams(const tdes_msg *d_msgs, size_t n_msgs,
                                        const void *d_schedules, size_t n_schedules,
                                        const void *d_in_base, size_t in_bytes,
                                        void *const *d_out_bases, size_t out_bytes,
                                        void *const *d_workspaces, size_t workspace_bytes,
                                        void *const *streams, int n_streams, int reps,
                                        tdes_batch_config *best);

/* The tuning cache file itself (host only, no device needed).  Load: the
 * entry for `device` (an architecture name such as "gfx950:sramecc+:xnack-")
 * and `cus` compute units from the JSON file at path into *out; returns 1
 * if found and valid, 0 if the file or the entry is missing or unreadable,
 * a negative tdes_status for bad arguments.  Save: write or replace that
 * entry (us_per_batch is recorded beside it), keeping the file's other
 * entries; the file is replaced atomically and its directory created.
 * Errors: TDES_ERR_ARG (NULL or empty path, a device name with quotes,
 * backslashes or control characters, an invalid configuration),
 * TDES_ERR_DEVICE (the file could not be written). */
int tdes_batch_config_load(const char *path, const char *device, uint32_t cus,
                           tdes_batch_config *out);
tdes_status tdes_batch_config_save(const char *path, const char *device, uint32_t cus,
                                   const tdes_batch_config *cfg, double us_per_batch);

/* The key material a launch of `kernel` (TDES_KERNEL_BITSLICE or
 * TDES_KERNEL_SPBOX; AUTO gives the bitsliced kernel's, its choice above
 * 1.5 times the table kernel's one-pass size) would receive for
 * schedule ks and direction dir, copied to host memory `out` (cap bytes).
 * Returns the number of bytes written, or a negative tdes_status
 * (TDES_ERR_ARG for NULL pointers, bad enums or cap too small).  For
 * inspection and testing: the encryption calls build it themselves. */
long tdes_kernel_key_bytes(const tdes_schedule *ks, int dir, int kernel, void *out, size_t cap);

/* Message of the last failed call on this thread ("" if none).  The
 * pointer stays valid until the next library call on this thread. */
const char *tdes_last_error(void);

/* TDES_ABI_VERSION of the built library. */
int tdes_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TDES_H */
