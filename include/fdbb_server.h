/*
 * fdbb_server.h -- native request server over the building blocks of fdbb.h.
 *
 * Requests are fdbb_task records (fdbb.h) whose outputs the server places:
 * the caller fills op, dim, dtype, dir, gamma, n and the input pointers; the
 * output pointers and leading dimensions are ignored on submission.  A
 * scheduler thread admits queued requests in arrival order while a launch
 * slot is free and their outputs fit in the server's device arena (the HBM
 * budget), runs every request admitted into a slot as one persistent batch
 * launch (FDBB_SERVE_BATCHED: continuous batching, one stream per slot,
 * launched with the configuration of fdbb_set_server_batch_config) or
 * each as its own launch on one stream (FDBB_SERVE_SINGLE: the
 * one-launch-per-request baseline), and reports a request complete when its
 * launch's completion event fires.  Outputs stay in the arena, with the
 * leading dimension n rounded up to 64 points, until fdbb_server_release.
 *
 * Ownership: the server owns its arena, streams, events and batch plans;
 * inputs belong to the caller, must hold their final values when the
 * request is submitted (the server's streams are not ordered after the
 * caller's work: synchronise first) and must stay valid until the request
 * completes.  Tags identify requests from submission to release and must be
 * unique among them.  All calls return fdbb_status codes and are
 * thread-safe; results are unaffected by which other requests share a
 * launch.  While launches are in flight the scheduler thread polls their
 * events without sleeping (one host core); idle, it sleeps until a
 * submission or a release.
 */
#ifndef FDBB_SERVER_H
#define FDBB_SERVER_H

#include <stdint.h>

#include "fdbb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { FDBB_SERVE_BATCHED = 0, FDBB_SERVE_SINGLE = 1 } fdbb_serve_mode;

typedef struct fdbb_server fdbb_server;

typedef struct {
    uint64_t tag;            /* the submitter's tag */
    int32_t status;          /* FDBB_OK, or FDBB_EHIP if its launch failed */
    int32_t pad;
    void *out0, *out1, *out2; /* outputs in the arena (NULL where unused) */
    int64_t ld;              /* leading dimension of every output */
    int64_t t_submit_ns, t_admit_ns, t_done_ns; /* steady clock */
} fdbb_completion;

typedef struct {
    int64_t submitted, completed, launches, errors;
    int64_t arena_bytes;      /* held by admitted or unreleased outputs */
    int64_t peak_arena_bytes;
    int64_t queued;
} fdbb_server_stats;

/* Create a server on the current device: a device arena of budget_bytes
 * (FDBB_ENOMEM if it cannot be allocated), `slots` launch slots (batches
 * in flight; in FDBB_SERVE_SINGLE mode, launches in flight on the one
 * stream), at most max_batch requests and max_batch_bytes moved HBM bytes
 * per batched launch (a request larger than that runs alone). */
int fdbb_server_create(int64_t budget_bytes, int slots, int max_batch, double max_batch_bytes, int mode,
                       fdbb_server **server);

/* Queue one request (validated as its single-call entry point would be;
 * FDBB_EINVAL for a tag still in use or an op the server does not run
 * (eigenvectors, char_apply); FDBB_ENOMEM if its outputs exceed the whole
 * arena). */
int fdbb_server_submit(fdbb_server *server, const fdbb_task *task, uint64_t tag);

/* Up to `max` completions, oldest first; *count gets how many. */
int fdbb_server_poll(fdbb_server *server, fdbb_completion *out, int max, int *count);

/* Give a completed request's outputs back to the arena and free its tag
 * (FDBB_EINVAL if the tag names no completed, unreleased request). */
int fdbb_server_release(fdbb_server *server, uint64_t tag);

int fdbb_server_get_stats(fdbb_server *server, fdbb_server_stats *stats);

/* Stop the scheduler, wait for launches in flight, free everything. */
int fdbb_server_destroy(fdbb_server *server);

#ifdef __cplusplus
}
#endif

#endif /* FDBB_SERVER_H */
