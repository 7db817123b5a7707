// C-ABI entry points of libtdes (declared in include/tdes.h): argument
// checks, key formats, kernel dispatch, error reporting.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "internal.h"

namespace {

thread_local std::string g_last_error;

tdes_status fail(tdes_status st, const char *fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

// Checks shared by every call that takes a device in/out buffer pair.
tdes_status check_buffers(const void *in, const void *out, size_t nbytes) {
    if (nbytes % 8 != 0)
        return fail(TDES_ERR_LENGTH, "length %zu is not a multiple of the 8-byte block", nbytes);
    if (nbytes == 0) return TDES_OK;
    if (in == nullptr || out == nullptr) return fail(TDES_ERR_ARG, "NULL data pointer");
    const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
    if ((a | b) % 8 != 0) return fail(TDES_ERR_ALIGN, "data pointers must be 8-byte aligned");
    if (a != b && a < b + nbytes && b < a + nbytes)
        return fail(TDES_ERR_OVERLAP, "input and output overlap without being identical");
    return TDES_OK;
}

// Checks shared by the batched calls (n_msgs > 0), on everything but the
// workspace.
tdes_status batch_checks(const tdes_msg *d_msgs, size_t n_msgs, const void *d_schedules,
                         size_t n_schedules, const void *d_in_base, const void *d_out_base) {
    if (d_msgs == nullptr || d_schedules == nullptr || d_in_base == nullptr ||
        d_out_base == nullptr)
        return fail(TDES_ERR_ARG, "NULL pointer");
    if (n_schedules == 0) return fail(TDES_ERR_ARG, "no schedules");
    if (n_schedules > TDES_BATCH_MAX_SCHEDULES)
        return fail(TDES_ERR_ARG, "%zu schedules: at most %u per batch", n_schedules,
                    (unsigned)TDES_BATCH_MAX_SCHEDULES);
    if (n_msgs > TDES_BATCH_MAX_MSGS)
        return fail(TDES_ERR_ARG, "%zu messages: at most %u per batch", n_msgs,
                    (unsigned)TDES_BATCH_MAX_MSGS);
    if (((uintptr_t)d_msgs | (uintptr_t)d_in_base | (uintptr_t)d_out_base) % 8 != 0 ||
        (uintptr_t)d_schedules % 16 != 0)
        return fail(TDES_ERR_ALIGN, "misaligned pointer");
    return TDES_OK;
}

// The checks above plus the caller's workspace.
tdes_status tdes_batch_submit_checks(const tdes_msg *d_msgs, size_t n_msgs, const void *d_schedules,
                                     size_t n_schedules, const void *d_in_base,
                                     const void *d_out_base, const void *d_workspace,
                                     size_t workspace_bytes) {
    if (d_workspace == nullptr) return fail(TDES_ERR_ARG, "NULL pointer");
    tdes_status st = batch_checks(d_msgs, n_msgs, d_schedules, n_schedules, d_in_base, d_out_base);
    if (st != TDES_OK) return st;
    if (workspace_bytes < tdes::batch_workspace_bytes(n_msgs))
        return fail(TDES_ERR_ARG, "workspace too small (%zu < %zu bytes)", workspace_bytes,
                    tdes::batch_workspace_bytes(n_msgs));
    if ((uintptr_t)d_workspace % 8 != 0) return fail(TDES_ERR_ALIGN, "misaligned pointer");
    return TDES_OK;
}

}  // namespace

tdes_status tdes::set_last_error(tdes_status st, const char *msg) {
    g_last_error = msg;
    return st;
}

int tdes::auto_kernel(size_t nbytes) {
    // one and a half passes: up to there the table kernel's launch is the
    // shorter (measured: 28.6 against 35.1 us at 6 MiB on 256 CUs, 35.6
    // against 35.2 at 6.5 MiB)
    return nbytes <= spbox_one_pass_bytes() / 2 * 3 ? TDES_KERNEL_SPBOX : TDES_KERNEL_BITSLICE;
}

hipError_t tdes::launch_ecb_auto(const tdes_schedule &ks, int dir, const uint8_t *in,
                                 uint8_t *out, size_t nbytes, hipStream_t stream) {
    if (auto_kernel(nbytes) == TDES_KERNEL_SPBOX) {
        RoundSequence seq;
        round_sequence(ks, dir, &seq);
        SpboxKeys k;
        spbox_keys(seq, &k);
        return launch_spbox(k, in, out, nbytes, stream);
    }
    BitsliceKeys k;
    bitslice_keys(ks, dir, &k);
    return launch_bitslice(k, in, out, nbytes, stream);
}

extern "C" {

tdes_status tdes_key_schedule(const uint8_t key24[24], tdes_schedule *out) {
    g_last_error.clear();
    if (key24 == nullptr || out == nullptr) return fail(TDES_ERR_ARG, "NULL key or schedule");
    for (int b = 0; b < 3; b++) tdes::des_round_keys(key24 + 8 * b, out->k[b]);  // Sec. III-A
    return TDES_OK;
}

int tdes_ecb_auto_kernel(size_t nbytes) {
    g_last_error.clear();
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(TDES_ERR_DEVICE, "no device");
    return tdes::auto_kernel(nbytes);
}

tdes_status tdes_ecb_crypt(const tdes_schedule *ks, int dir, int kernel, const void *d_in,
                           void *d_out, size_t nbytes, void *stream) {
    g_last_error.clear();
    if (ks == nullptr) return fail(TDES_ERR_ARG, "NULL schedule");
    if (dir != TDES_ENCRYPT && dir != TDES_DECRYPT) return fail(TDES_ERR_ARG, "bad direction %d", dir);
    if (kernel < TDES_KERNEL_AUTO || kernel > TDES_KERNEL_SPBOX)
        return fail(TDES_ERR_ARG, "bad kernel %d", kernel);
    tdes_status st = check_buffers(d_in, d_out, nbytes);
    if (st != TDES_OK || nbytes == 0) return st;

    const uint8_t *in = static_cast<const uint8_t *>(d_in);
    uint8_t *out = static_cast<uint8_t *>(d_out);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (kernel == TDES_KERNEL_SPBOX) {
        tdes::RoundSequence seq;
        tdes::round_sequence(*ks, dir, &seq);
        tdes::SpboxKeys k;
        tdes::spbox_keys(seq, &k);
        e = tdes::launch_spbox(k, in, out, nbytes, s);
    } else if (kernel == TDES_KERNEL_BITSLICE) {
        tdes::BitsliceKeys k;
        tdes::bitslice_keys(*ks, dir, &k);
        e = tdes::launch_bitslice(k, in, out, nbytes, s);
    } else {
        e = tdes::launch_ecb_auto(*ks, dir, in, out, nbytes, s);
    }
    if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return TDES_OK;
}

tdes_status tdes_ctr_crypt(const tdes_schedule *ks, const uint8_t iv[8], const void *d_in,
                           void *d_out, size_t nbytes, void *stream) {
    g_last_error.clear();
    if (ks == nullptr || iv == nullptr) return fail(TDES_ERR_ARG, "NULL schedule or iv");
    tdes_status st = check_buffers(d_in, d_out, nbytes);
    if (st != TDES_OK || nbytes == 0) return st;
    uint64_t ctr = 0;
    for (int i = 0; i < 8; i++) ctr = ctr << 8 | iv[i];  // big-endian counter value
    tdes::BitsliceKeys k;
    tdes::bitslice_keys(*ks, TDES_ENCRYPT, &k);
    hipError_t e = tdes::launch_bitslice_ctr(k, ctr, static_cast<const uint8_t *>(d_in),
                                             static_cast<uint8_t *>(d_out), nbytes,
                                             static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return TDES_OK;
}

tdes_status tdes_cbc_decrypt(const tdes_schedule *ks, const uint8_t iv[8], const void *d_in,
                             void *d_out, size_t nbytes, void *stream) {
    g_last_error.clear();
    if (ks == nullptr || iv == nullptr) return fail(TDES_ERR_ARG, "NULL schedule or iv");
    tdes_status st = check_buffers(d_in, d_out, nbytes);
    if (st != TDES_OK || nbytes == 0) return st;
    if (d_in == d_out)
        return fail(TDES_ERR_OVERLAP, "CBC decryption re-reads the ciphertext: no in-place");
    const uint32_t iv0 = iv[0] | iv[1] << 8 | iv[2] << 16 | (uint32_t)iv[3] << 24;
    const uint32_t iv1 = iv[4] | iv[5] << 8 | iv[6] << 16 | (uint32_t)iv[7] << 24;
    tdes::BitsliceKeys k;
    tdes::bitslice_keys(*ks, TDES_DECRYPT, &k);
    hipError_t e = tdes::launch_bitslice_cbc_dec(k, iv0, iv1, static_cast<const uint8_t *>(d_in),
                                                 static_cast<uint8_t *>(d_out), nbytes,
                                                 static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return TDES_OK;
}

tdes_status tdes_ecb_paper_design(const tdes_schedule *ks, int dir, const void *d_in, void *d_out,
                                  size_t nbytes, void *stream) {
    g_last_error.clear();
    if (ks == nullptr) return fail(TDES_ERR_ARG, "NULL schedule");
    if (dir != TDES_ENCRYPT && dir != TDES_DECRYPT) return fail(TDES_ERR_ARG, "bad direction %d", dir);
    tdes_status st = check_buffers(d_in, d_out, nbytes);
    if (st != TDES_OK || nbytes == 0) return st;
    // The three passes in order, as (base key, decrypt?): E_K1, D_K2, E_K3;
    // decryption D_K3, E_K2, D_K1 (Sec. III-B).  A decrypting pass takes the
    // round keys in reverse (Sec. IV-B: reversed on the host).
    const int key_of[2][3] = {{0, 1, 2}, {2, 1, 0}};
    const bool dec_of[2][3] = {{false, true, false}, {true, false, true}};
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int pass = 0; pass < 3; pass++) {
        tdes::ReplicaKeyBits kb;
        const uint64_t *rk = ks->k[key_of[dir][pass]];
        for (int i = 0; i < 16; i++) {
            const uint64_t key = rk[dec_of[dir][pass] ? 15 - i : i];
            for (int j = 0; j < 48; j++) kb.k[48 * i + j] = (uint8_t)((key >> (47 - j)) & 1);
        }
        hipError_t e = tdes::launch_replica_pass(kb, pass == 0 ? static_cast<const uint8_t *>(d_in)
                                                               : static_cast<const uint8_t *>(d_out),
                                                 static_cast<uint8_t *>(d_out), nbytes, s);
        if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    }
    return TDES_OK;
}

tdes_status tdes_ecb_encrypt(const tdes_schedule *ks, const void *d_in, void *d_out,
                             size_t nbytes, void *stream) {
    return tdes_ecb_crypt(ks, TDES_ENCRYPT, TDES_KERNEL_AUTO, d_in, d_out, nbytes, stream);
}

tdes_status tdes_ecb_decrypt(const tdes_schedule *ks, const void *d_in, void *d_out,
                             size_t nbytes, void *stream) {
    return tdes_ecb_crypt(ks, TDES_DECRYPT, TDES_KERNEL_AUTO, d_in, d_out, nbytes, stream);
}

tdes_status tdes_schedule_upload(const tdes_schedule *h, size_t n, void *d_dst, void *stream) {
    g_last_error.clear();
    if (n == 0) return TDES_OK;
    if (h == nullptr || d_dst == nullptr) return fail(TDES_ERR_ARG, "NULL schedules or destination");
    if ((uintptr_t)d_dst % 16 != 0) return fail(TDES_ERR_ALIGN, "destination must be 16-byte aligned");
    std::vector<uint32_t> words(n * tdes::kDeviceScheduleWords);
    for (size_t i = 0; i < n; i++)
        tdes::device_schedule_words(h[i], words.data() + i * tdes::kDeviceScheduleWords);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(d_dst, words.data(), words.size() * sizeof(uint32_t),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "schedule upload failed: %s", hipGetErrorString(e));
    return TDES_OK;
}

tdes_status tdes_schedule_expand(const void *d_keys24, size_t n, void *d_schedules, void *stream) {
    g_last_error.clear();
    if (n == 0) return TDES_OK;
    if (d_keys24 == nullptr || d_schedules == nullptr) return fail(TDES_ERR_ARG, "NULL pointer");
    if ((uintptr_t)d_schedules % 16 != 0) return fail(TDES_ERR_ALIGN, "schedules must be 16-byte aligned");
    hipError_t e = tdes::launch_expand(static_cast<const uint8_t *>(d_keys24), n,
                                       static_cast<uint32_t *>(d_schedules),
                                       static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "expand launch failed: %s", hipGetErrorString(e));
    return TDES_OK;
}

tdes_status tdes_ecb_host(const tdes_schedule *ks, int dir, const void *h_in, void *h_out,
                          size_t nbytes, void *d_work, size_t work_bytes, size_t chunk_bytes) {
    g_last_error.clear();
    if (ks == nullptr) return fail(TDES_ERR_ARG, "NULL schedule");
    if (dir != TDES_ENCRYPT && dir != TDES_DECRYPT) return fail(TDES_ERR_ARG, "bad direction %d", dir);
    tdes_status st = check_buffers(h_in, h_out, nbytes);
    if (st != TDES_OK || nbytes == 0) return st;
    tdes::BitsliceKeys k;
    if (d_work == nullptr) {  // direct: the kernel works on the mapped host buffers
        uint8_t *d_in = nullptr, *d_out = nullptr;
        hipError_t e = tdes::mapped_range(h_in, nbytes, &d_in);
        if (e == hipSuccess) e = tdes::mapped_range(h_out, nbytes, &d_out);
        if (e != hipSuccess)
            return fail(TDES_ERR_ARG, "direct mode needs pinned host buffers: %s", hipGetErrorString(e));
        tdes::bitslice_keys(*ks, dir, &k);
        e = tdes::run_host_direct(k, d_in, d_out, nbytes);
        if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "direct host run failed: %s", hipGetErrorString(e));
        return TDES_OK;
    }
    if (chunk_bytes == 0) return fail(TDES_ERR_ARG, "chunk_bytes is 0");
    if (chunk_bytes % 8 != 0)
        return fail(TDES_ERR_LENGTH, "chunk_bytes %zu is not a multiple of 8", chunk_bytes);
    if ((uintptr_t)d_work % 256 != 0) return fail(TDES_ERR_ALIGN, "workspace must be 256-byte aligned");
    if (work_bytes < chunk_bytes)
        return fail(TDES_ERR_ARG, "workspace (%zu bytes) smaller than one chunk (%zu)", work_bytes,
                    chunk_bytes);
    size_t n_slots = work_bytes / chunk_bytes;
    if (n_slots > TDES_HOST_MAX_SLOTS) n_slots = TDES_HOST_MAX_SLOTS;
    tdes::bitslice_keys(*ks, dir, &k);
    hipError_t e = tdes::run_host_pipeline(k, static_cast<const uint8_t *>(h_in),
                                           static_cast<uint8_t *>(h_out), nbytes,
                                           static_cast<uint8_t *>(d_work), n_slots, chunk_bytes);
    if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "host pipeline failed: %s", hipGetErrorString(e));
    return TDES_OK;
}

size_t tdes_batch_workspace_bytes(size_t n_msgs) { return tdes::batch_workspace_bytes(n_msgs); }

tdes_status tdes_batch_submit(const tdes_msg *d_msgs, size_t n_msgs, const void *d_schedules,
                              size_t n_schedules, const void *d_in_base, size_t in_bytes,
                              void *d_out_base, size_t out_bytes, void *d_workspace,
                              size_t workspace_bytes, void *stream) {
    g_last_error.clear();
    if (n_msgs == 0) return TDES_OK;
    tdes_status st = tdes_batch_submit_checks(d_msgs, n_msgs, d_schedules, n_schedules, d_in_base,
                                              d_out_base, d_workspace, workspace_bytes);
    if (st != TDES_OK) return st;
    hipError_t e = tdes::launch_batch(d_msgs, n_msgs, static_cast<const uint32_t *>(d_schedules),
                                      n_schedules, static_cast<const uint8_t *>(d_in_base),
                                      in_bytes, static_cast<uint8_t *>(d_out_base), out_bytes,
                                      static_cast<uint64_t *>(d_workspace), nullptr,
                                      static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "batch launch failed: %s", hipGetErrorString(e));
    return TDES_OK;
}

tdes_status tdes_batch_submit_noalloc(const tdes_msg *d_msgs, size_t n_msgs,
                                      const void *d_schedules, size_t n_schedules,
                                      const void *d_in_base, size_t in_bytes, void *d_out_base,
                                      size_t out_bytes, uint64_t *d_skipped, void *stream) {
    g_last_error.clear();
    if (n_msgs == 0) return TDES_OK;
    if (n_msgs > TDES_BATCH_NOALLOC_MAX_MSGS)
        return fail(TDES_ERR_ARG, "%zu messages: at most %u per call without a workspace", n_msgs,
                    (unsigned)TDES_BATCH_NOALLOC_MAX_MSGS);
    tdes_status st = batch_checks(d_msgs, n_msgs, d_schedules, n_schedules, d_in_base, d_out_base);
    if (st != TDES_OK) return st;
    if ((uintptr_t)d_skipped % 8 != 0) return fail(TDES_ERR_ALIGN, "misaligned pointer");
    uint64_t *ws = nullptr;
    size_t ws_bytes = 0;
    hipError_t e = tdes::noalloc_workspace(&ws, &ws_bytes);
    if (e != hipSuccess)
        return fail(TDES_ERR_DEVICE, "no-alloc workspace: %s", hipGetErrorString(e));
    if (ws_bytes < tdes::batch_workspace_bytes(n_msgs))  // guarded by the limit above
        return fail(TDES_ERR_ARG, "no-alloc workspace too small");
    e = tdes::launch_batch(d_msgs, n_msgs, static_cast<const uint32_t *>(d_schedules), n_schedules,
                           static_cast<const uint8_t *>(d_in_base), in_bytes,
                           static_cast<uint8_t *>(d_out_base), out_bytes, ws, d_skipped,
                           static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "batch launch failed: %s", hipGetErrorString(e));
    return TDES_OK;
}

tdes_status tdes_batch_autotune(const tdes_msg *d_msgs, size_t n_msgs, const void *d_schedules,
                                size_t n_schedules, const void *d_in_base, size_t in_bytes,
                                void *d_out_base, size_t out_bytes, void *d_workspace,
                                size_t workspace_bytes, void *stream, int reps,
                                tdes_batch_config *best) {
    void *outs[1] = {d_out_base}, *wss[1] = {d_workspace}, *streams[1] = {stream};
    return tdes_batch_autotune_streams(d_msgs, n_msgs, d_schedules, n_schedules, d_in_base,
                                       in_bytes, outs, out_bytes, wss, workspace_bytes, streams, 1,
                                       reps, best);
}

tdes_status tdes_batch_autotune_streams(const tdes_msg *d_msgs, size_t n_msgs,
                                        const void *d_schedules, size_t n_schedules,
                                        const void *d_in_base, size_t in_bytes,
                                        void *const *d_out_bases, size_t out_bytes,
                                        void *const *d_workspaces, size_t workspace_bytes,
                                        void *const *streams, int n_streams, int reps,
                                        tdes_batch_config *best) {
    g_last_error.clear();
    if (reps < 1 || best == nullptr) return fail(TDES_ERR_ARG, "reps must be >= 1 and best non-NULL");
    if (n_streams < 1 || n_streams > tdes::kMaxTuneLanes)
        return fail(TDES_ERR_ARG, "n_streams must be 1..%d", tdes::kMaxTuneLanes);
    if (d_out_bases == nullptr || d_workspaces == nullptr || streams == nullptr)
        return fail(TDES_ERR_ARG, "NULL lane array");
    if (n_msgs == 0) return fail(TDES_ERR_ARG, "nothing to tune on: no messages");
    tdes::TuneLane lanes[tdes::kMaxTuneLanes];
    auto overlap = [](uintptr_t a, size_t na, uintptr_t b, size_t nb) {
        return na > 0 && nb > 0 && a < b + nb && b < a + na;
    };
    for (int i = 0; i < n_streams; i++) {
        // same checks as tdes_batch_submit, for every lane
        tdes_status st = tdes_batch_submit_checks(d_msgs, n_msgs, d_schedules, n_schedules,
                                                  d_in_base, d_out_bases[i], d_workspaces[i],
                                                  workspace_bytes);
        if (st != TDES_OK) return st;
        // every trial rewrites the output from the input: they must not
        // alias, or each trial would encrypt the previous trial's result again
        if (overlap((uintptr_t)d_in_base, in_bytes, (uintptr_t)d_out_bases[i], out_bytes))
            return fail(TDES_ERR_OVERLAP,
                        "autotuning runs the batch several times: input and output must not overlap");
        for (int j = 0; j < i; j++) {
            // lanes run at the same time: their outputs and workspaces are their own
            if (overlap((uintptr_t)d_out_bases[i], out_bytes, (uintptr_t)d_out_bases[j], out_bytes))
                return fail(TDES_ERR_OVERLAP, "the lanes' outputs overlap");
            if (overlap((uintptr_t)d_workspaces[i], workspace_bytes, (uintptr_t)d_workspaces[j],
                        workspace_bytes))
                return fail(TDES_ERR_OVERLAP, "the lanes' workspaces overlap");
        }
        lanes[i] = {static_cast<uint8_t *>(d_out_bases[i]), static_cast<uint64_t *>(d_workspaces[i]),
                    static_cast<hipStream_t>(streams[i])};
    }
    tdes::BatchConfig c;
    float us = 0;
    hipError_t e = tdes::batch_autotune(d_msgs, n_msgs, static_cast<const uint32_t *>(d_schedules),
                                        n_schedules, static_cast<const uint8_t *>(d_in_base),
                                        in_bytes, lanes, n_streams, out_bytes, reps, &c, &us);
    if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "autotune failed: %s", hipGetErrorString(e));
    best->kmax = (uint32_t)c.kmax;
    best->waves = (uint32_t)c.waves;
    best->grid_mult = (uint32_t)c.grid_mult;
    best->saved = (!tdes::tune_cache_path().empty() && tdes::batch_config_persist(c, us)) ? 1u : 0u;
    return TDES_OK;
}

tdes_status tdes_batch_get_config(tdes_batch_config *out) {
    g_last_error.clear();
    if (out == nullptr) return fail(TDES_ERR_ARG, "NULL config");
    tdes::BatchConfig c;
    hipError_t e = tdes::batch_config_current(&c);
    if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "no device: %s", hipGetErrorString(e));
    out->kmax = (uint32_t)c.kmax;
    out->waves = (uint32_t)c.waves;
    out->grid_mult = (uint32_t)c.grid_mult;
    out->saved = 0;
    return TDES_OK;
}

namespace {
bool to_config(const tdes_batch_config *cfg, tdes::BatchConfig *c) {
    if (cfg == nullptr || cfg->kmax > 64 || cfg->waves > 64 || cfg->grid_mult > 64) return false;
    *c = tdes::BatchConfig{(int)cfg->kmax, (int)cfg->waves, (int)cfg->grid_mult};
    return tdes::batch_config_valid(*c);
}
}  // namespace

tdes_status tdes_batch_set_config(const tdes_batch_config *cfg) {
    g_last_error.clear();
    tdes::BatchConfig c;
    if (!to_config(cfg, &c)) return fail(TDES_ERR_ARG, "not a compiled batched-kernel configuration");
    hipError_t e = tdes::batch_config_set(c);
    if (e != hipSuccess) return fail(TDES_ERR_DEVICE, "no device: %s", hipGetErrorString(e));
    return TDES_OK;
}

int tdes_batch_config_load(const char *path, const char *device, uint32_t cus,
                           tdes_batch_config *out) {
    g_last_error.clear();
    if (path == nullptr || *path == '\0' || device == nullptr || out == nullptr)
        return fail(TDES_ERR_ARG, "NULL or empty argument");
    tdes::BatchConfig c;
    const int r = tdes::cache_load(path, device, (long)cus, &c);
    if (r < 0) return fail(TDES_ERR_ARG, "bad device name");
    if (r == 1) {
        out->kmax = (uint32_t)c.kmax;
        out->waves = (uint32_t)c.waves;
        out->grid_mult = (uint32_t)c.grid_mult;
        out->saved = 0;
    }
    return r;
}

tdes_status tdes_batch_config_save(const char *path, const char *device, uint32_t cus,
                                   const tdes_batch_config *cfg, double us_per_batch) {
    g_last_error.clear();
    tdes::BatchConfig c;
    if (path == nullptr || *path == '\0' || device == nullptr || !to_config(cfg, &c))
        return fail(TDES_ERR_ARG, "NULL or empty argument, or not a compiled configuration");
    if (strchr(device, '"') || strchr(device, '\\') || *device == '\0')
        return fail(TDES_ERR_ARG, "bad device name");
    for (const char *p = device; *p; p++)
        if ((unsigned char)*p < 0x20) return fail(TDES_ERR_ARG, "bad device name");
    if (!tdes::cache_save(path, device, (long)cus, c, us_per_batch))
        return fail(TDES_ERR_DEVICE, "could not write %s", path);
    return TDES_OK;
}

long tdes_kernel_key_bytes(const tdes_schedule *ks, int dir, int kernel, void *out, size_t cap) {
    g_last_error.clear();
    if (ks == nullptr || out == nullptr) return fail(TDES_ERR_ARG, "NULL schedule or buffer");
    if (dir != TDES_ENCRYPT && dir != TDES_DECRYPT) return fail(TDES_ERR_ARG, "bad direction %d", dir);
    if (kernel < TDES_KERNEL_AUTO || kernel > TDES_KERNEL_SPBOX)
        return fail(TDES_ERR_ARG, "bad kernel %d", kernel);
    tdes::RoundSequence seq;
    tdes::round_sequence(*ks, dir, &seq);
    if (kernel == TDES_KERNEL_SPBOX) {
        tdes::SpboxKeys k;
        if (cap < sizeof k) return fail(TDES_ERR_ARG, "buffer too small (%zu < %zu)", cap, sizeof k);
        tdes::spbox_keys(seq, &k);
        memcpy(out, &k, sizeof k);
        return (long)sizeof k;
    }
    tdes::BitsliceKeys k;
    if (cap < sizeof k) return fail(TDES_ERR_ARG, "buffer too small (%zu < %zu)", cap, sizeof k);
    tdes::bitslice_keys(*ks, dir, &k);
    memcpy(out, &k, sizeof k);
    return (long)sizeof k;
}

const char *tdes_last_error(void) { return g_last_error.c_str(); }

int tdes_abi_version(void) { return TDES_ABI_VERSION; }

}  // extern "C"
