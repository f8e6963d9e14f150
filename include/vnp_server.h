/*
 * vnp request server: continuous batching of norm requests on one GPU.
 *
 * Serves the single-vector calls of vnp.h (xNRMF / xNRMP of Novakovic, arXiv 2509.06220,
 * Sect. 1, 3, 4) to many concurrent clients.  Admission by device memory, two ways:
 *   - vnp_server_submit_copy: the server copies the payload into a block of its pool when
 *     it admits the request (in arrival order) and frees the block when the request
 *     completes; while the pool cannot hold the next request, it and every later one wait
 *     (back-pressure, counted in the statistics);
 *   - vnp_server_alloc + vnp_server_submit: the caller writes the payload into a pool
 *     block it holds (VNP_EAGAIN when the pool is full) or names any device memory.
 * A batcher thread collects the admitted requests and launches them as one batched launch
 * per (dtype, p) class on one of `streams` HIP streams; requests that arrive while
 * batches are running start in the next batch on a free stream, so their work overlaps
 * on the device.  Each result is bitwise equal to the single-vector call on the same data
 * (same canonical tree), alone or in any mix.
 *
 * Threads: the batcher and one completion thread per stream.  While idle, each polls for
 * new work for up to 200 microseconds before it blocks, so an active server keeps up to
 * streams + 1 host cores busy for that long after its last request.
 *
 * Conventions as in vnp.h: 0 = success, -k = argument k invalid, > 0 = HIP error or one
 * of VNP_EAGAIN / VNP_ENOTFOUND / VNP_EPENDING.  All functions are thread-safe.
 */
#ifndef VNP_SERVER_H
#define VNP_SERVER_H

#include <stdint.h>

#include "vnp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vnp_server vnp_server;

typedef struct {
    int64_t pool_bytes;    /* device memory pool for payloads (vnp_server_alloc) */
    int max_batch;         /* most requests in one batch (>= 1) */
    int streams;           /* HIP streams = batches that may be in flight at once (>= 1) */
    int max_wait_us;       /* while batches are in flight, a batch smaller than max_batch starts at
                              the latest when its oldest request has waited this long (an idle
                              device starts at once); 0 = as soon as a stream is free */
    int inject_failure_every; /* testing: treat every k-th batch as failed (0 = never); its
                                 requests are then rerun one per batch */
} vnp_server_config;

typedef struct {
    int dtype;        /* VNP_F64 or VNP_F32 */
    double p;         /* 2 = Frobenius; > 0, may be +inf */
    int64_t n;        /* elements */
    const void *x;    /* device address of the vector (pool or any device memory) */
    int64_t incx;     /* stride, BLAS convention, != 0 */
} vnp_request;

typedef struct {
    double value;        /* the norm (binary32 results are widened exactly) */
    int status;          /* 0, or the INFO code that rejected the request */
    int64_t t_submit_ns; /* vnp_server_clock_ns() at submission */
    int64_t t_done_ns;   /* vnp_server_clock_ns() when the result became available */
} vnp_result;

typedef struct {
    int64_t submitted, completed, rejected, batches, launches, failed_batches;
    int64_t max_batch_seen, pool_free_bytes, pool_bytes, pending, in_flight;
    int64_t host_launch_ns;  /* total host time spent enqueueing batches */
    int64_t batch_ns;        /* total time from a batch's enqueue to its completion being seen */
    int64_t batch_ns_max;    /* longest such time */
    int64_t cancelled;       /* requests completed as VNP_ECANCELED by vnp_server_destroy */
    int64_t admission_waits; /* copy requests that found the pool full when first considered */
    int64_t admission_wait_ns;     /* their total wait for pool memory */
    int64_t admission_wait_ns_max; /* the longest such wait */
} vnp_server_stats;

/* Errors: srv == NULL -> -1; cfg invalid -> -2; > 0 HIP error (pool allocation). */
int vnp_server_create(vnp_server **srv, const vnp_server_config *cfg);
/* Finishes the batches in flight; requests not yet launched complete with status
 * VNP_ECANCELED (value NaN).  Threads blocked in vnp_server_wait return their ticket's
 * result before the server is freed; no call may start on srv once destroy has begun.
 * Then frees the pool and the server. */
int vnp_server_destroy(vnp_server *srv);

/* Device memory from the pool (256-byte aligned).  VNP_EAGAIN if no free block is large
 * enough right now.  Errors: srv NULL -> -1; bytes <= 0 -> -2; dptr NULL -> -3. */
int vnp_server_alloc(vnp_server *srv, int64_t bytes, void **dptr);
/* Returns a block to the pool.  Errors: -1, -2 (not a live pool block). */
int vnp_server_free(vnp_server *srv, void *dptr);

/* Queues a request; *ticket identifies it.  An invalid request is accepted and completes
 * at once with its INFO code in vnp_result.status (n < 0 or > VNP_MAX_N -> -3, x NULL ->
 * -4, incx == 0 -> -5, p invalid for the request's dtype (as in vnp.h) -> -2, unknown
 * dtype -> -1).  The payload must stay valid until the request completes.  Errors of the
 * call: srv NULL -> -1; req NULL -> -2; ticket NULL -> -3. */
int vnp_server_submit(vnp_server *srv, const vnp_request *req, uint64_t *ticket);
/* As vnp_server_submit, but req->x is the caller's copy of the payload (device memory or
 * host-mapped pinned memory, n elements with stride incx), which the server copies into a
 * pool block of n elements when it admits the request; the norm is computed on that block
 * (the same bits as on req->x).  req->x must stay valid until the request completes.
 * Requests wait in arrival order while the pool cannot hold the next one; a request larger
 * than the whole pool completes at once with status VNP_ENOMEM.  Errors as
 * vnp_server_submit. */
int vnp_server_submit_copy(vnp_server *srv, const vnp_request *req, uint64_t *ticket);
/* Non-blocking: 0 and *out filled (and the ticket released) if done, else VNP_EPENDING;
 * VNP_ENOTFOUND for an unknown or already released ticket. */
int vnp_server_poll(vnp_server *srv, uint64_t ticket, vnp_result *out);
/* Blocking up to timeout_us (< 0: no limit); same results as poll. */
int vnp_server_wait(vnp_server *srv, uint64_t ticket, int64_t timeout_us, vnp_result *out);

int vnp_server_get_stats(vnp_server *srv, vnp_server_stats *st);
/* The server's monotonic clock, nanoseconds. */
int64_t vnp_server_clock_ns(void);

#ifdef __cplusplus
}
#endif

#endif /* VNP_SERVER_H */
