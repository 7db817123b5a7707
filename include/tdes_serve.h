/*
 * tdes_serve.h - a request server around the batched 3DES-EDE ECB path.
 *
 * Requests (a key bundle, a direction and a device input) are queued by
 * tdes_server_submit and turned into batches by tdes_server_progress:
 * continuous batching over several HIP streams ("slots").  A request is
 * admitted, strictly in arrival order, when its input and output bytes fit
 * the in-flight budget and its output fits the caller's device arena;
 * admitted requests are packed into the next batch of a free slot (key
 * generation and the batched cipher run on the device, see tdes.h), so
 * requests that arrive while other batches run are admitted and launched as
 * slots and memory free up, and their work overlaps on the device.  A
 * request's result stays in the arena until tdes_server_release.
 *
 * Same conventions as tdes.h.  A server is used from one host thread at a
 * time.  The server allocates its staging buffers, streams and events once,
 * in tdes_server_create; submit / progress / release allocate no device
 * memory.
 */
#ifndef TDES_SERVE_H
#define TDES_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "tdes.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tdes_server tdes_server;

enum {
    TDES_SERVE_BATCHED = 0,   /* continuous batching over `slots` streams           */
    TDES_SERVE_PLAIN = 1,     /* reference: one plain launch per request, in
                                 arrival order, on one stream (host key schedule)   */
    TDES_SERVE_HOST_TEST = 2  /* no device work at all: a batch "completes" at the
                                 test_polls-th progress call counting the one that
                                 launched it (at least the next one); for tests of
                                 the scheduler                                       */
};

typedef struct {
    void *d_arena;            /* device memory for results, 256-byte aligned, owned by
                                 the caller; never dereferenced in HOST_TEST mode    */
    uint64_t arena_bytes;     /* its size                                           */
    uint64_t budget_bytes;    /* in-flight limit: sum over admitted, unreleased
                                 requests of input (until completion) + output
                                 (until release) bytes; 0 = 2 * arena_bytes         */
    uint32_t mode;            /* TDES_SERVE_*                                       */
    uint32_t slots;           /* batches in flight at once, 1..16                   */
    uint32_t max_batch_msgs;  /* requests per batch, 1..65536                       */
    uint32_t test_polls;      /* HOST_TEST: progress calls a batch takes (>= 2)     */
    uint64_t max_batch_bytes; /* payload bytes per batch (0 = no limit)             */
    uint32_t test_fail_batch; /* HOST_TEST: the launch of batch number
                                 test_fail_batch - 1 fails as a HIP launch error
                                 would (0 = never); for tests of the error path   */
    uint32_t reserved;        /* 0                                                   */
} tdes_server_config;

typedef struct {
    uint8_t key24[24];        /* K1 || K2 || K3                                      */
    uint32_t dir;             /* TDES_ENCRYPT / TDES_DECRYPT                         */
    uint32_t reserved;        /* 0                                                   */
    const void *d_in;         /* device input, 8-byte aligned, valid until completion */
    uint64_t nbytes;          /* multiple of 8                                        */
    uint64_t tag;             /* caller's id, returned in the completion              */
} tdes_request;               /* 56 bytes */

typedef struct {
    uint64_t tag;
    void *d_out;              /* result (nbytes) in the arena, until released          */
    uint64_t nbytes;
    int32_t status;           /* TDES_OK or a tdes_status                              */
    uint32_t batch;           /* sequence number of the batch that ran it             */
    double t_submit;          /* tdes_server_now() at submit, admission, launch and   */
    double t_admit;           /* when progress saw the batch finished                 */
    double t_launch;
    double t_done;
} tdes_completion;            /* 64 bytes */

typedef struct {
    uint64_t submitted, admitted, completed, released, rejected;
    uint64_t queued;          /* waiting for admission now                          */
    uint64_t in_flight_bytes, peak_in_flight_bytes;
    uint64_t arena_used_bytes, peak_arena_used_bytes;
    uint64_t batches, batched_msgs, batched_bytes;
    uint32_t busy_slots, peak_busy_slots;
    uint64_t failed;          /* completed with a device error (no result)          */
} tdes_server_stats;

/* Create a server.  Errors: TDES_ERR_ARG (bad config), TDES_ERR_ALIGN,
 * TDES_ERR_NOMEM / TDES_ERR_DEVICE (staging allocation failed). */
tdes_status tdes_server_create(const tdes_server_config *cfg, tdes_server **out);

/* Wait for all work in flight, then free the server's own resources (the
 * arena is the caller's). */
void tdes_server_destroy(tdes_server *s);

/* Queue n requests (copied).  A request that can never be admitted (bad
 * length or alignment, or larger than the budget or the arena) is not
 * queued: it completes at the next progress call with a nonzero status.
 * Errors: TDES_ERR_ARG (NULL). */
tdes_status tdes_server_submit(tdes_server *s, const tdes_request *reqs, size_t n);

/* Non-blocking step: retire finished batches, admit queued requests and
 * launch batches on free slots, then hand out up to cap completions
 * (*n_out of them).  If HIP reports an error for a batch (its launch, or
 * the query of its completion), every request of that batch completes with
 * status TDES_ERR_DEVICE and no result (d_out NULL, nothing to release):
 * its budget and arena space are given back at once, and tdes_last_error()
 * holds HIP's message.  Errors: TDES_ERR_ARG. */
tdes_status tdes_server_progress(tdes_server *s, tdes_completion *out, size_t cap, size_t *n_out);

/* Give back the arena space of a completed request (its d_out).
 * Errors: TDES_ERR_ARG if d_out is not a live result. */
tdes_status tdes_server_release(tdes_server *s, void *d_out);

/* tdes_server_release for n results at once (d_outs: n host-memory entries).
 * Every live entry is released, whatever the others are; *n_released (if
 * not NULL) receives how many were.  Errors: TDES_ERR_ARG for a NULL
 * argument or if any entry is not a live result (the message names the
 * first such entry). */
tdes_status tdes_server_release_many(tdes_server *s, void *const *d_outs, size_t n,
                                     size_t *n_released);

tdes_status tdes_server_get_stats(const tdes_server *s, tdes_server_stats *out);

/* The clock the completion times use (seconds, monotonic). */
double tdes_server_now(void);

#ifdef __cplusplus
}
#endif

#endif /* TDES_SERVE_H */
