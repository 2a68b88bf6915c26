/*
 * lbessel serving runtime: a request server in front of the lbessel kernels
 * (include/lbessel.h) for a stream of uneven requests, such as the Poisson
 * request streams of a metric-learning or inference service.
 *
 * Request types:
 *   - evaluation: n pairs (v, x) in HOST memory -> n log-values into host
 *     memory; kind 0 = log I_v(x), 1 = log K_v(x); precision 64 or 32.
 *     Pinned host memory (hipHostMalloc) lets the copies overlap compute;
 *     pageable memory works but serialises the server on each copy.
 *   - device-resident evaluation: the same with v, x and out in DEVICE
 *     memory (arrays a model on the same GPU produced or consumes): no
 *     copies, no arena data; the batch's segmented launch reads and writes
 *     the caller's arrays directly.
 *   - vMF fit: an n x p float32 feature matrix in DEVICE memory (typically
 *     the output of a model on the same GPU) -> the maximum-likelihood
 *     concentration, computed on the device (lbessel_vmf_fit_f32), into 4
 *     host doubles {kappa, R, kappa_0, Newton steps}.
 *
 * How requests flow (batched mode):
 *   1. submit: the request joins a FIFO queue; the call returns a ticket.
 *   2. admission by memory: the scheduler thread moves the queue head into
 *      the server's device arena as soon as a first-fit region of the size
 *      the request needs is free (inputs, outputs, workspace).  Admission
 *      is strictly FIFO, so a large request is never starved.
 *   3. continuous batching: whenever one of the server's streams is free,
 *      the admitted requests not yet launched form the next batch, in FIFO
 *      order up to the batch caps (a large evaluation request or a vMF fit
 *      goes out alone): its host inputs are copied in, all evaluation
 *      requests of one (kind, precision) run as ONE segmented launch
 *      (lbessel_eval_segments; up to LBESSEL_SEG_INLINE_MAX requests per
 *      launch with the segment table in the kernel arguments,
 *      lbessel_eval_segments_inline), vMF requests run their column-sum and
 *      Newton kernels, and the outputs are copied back.  Requests that
 *      arrive while batches are on the GPU are admitted as memory frees up
 *      and go out with the next batch; up to `streams` batches overlap
 *      (copies of one with kernels of another).
 *   4. completion: each request completes, and releases its arena region,
 *      as soon as the copy of its own results has finished (one event per
 *      request on the batch's stream).
 * Plain mode runs the same queue and admission but launches each request
 * on its own with the single-array entry points (one launch per request,
 * one request per stream): the baseline the batching is measured against.
 *
 * Every result is bit-identical to what the single-array entry point gives
 * for that request alone: each element's value depends on its own (v, x)
 * only, and the vMF reduction order is fixed.
 *
 * Threading: submit/wait/stats may be called from any host thread.  The
 * server owns one scheduler thread, its device arena (allocated at create)
 * and pinned staging for segment tables; the caller owns every request
 * buffer and must keep it valid and untouched until the request is done.
 */
#ifndef LBESSEL_SERVE_H
#define LBESSEL_SERVE_H

#include <stdint.h>

#include "lbessel.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBESSEL_ETOOBIG (-4)    /* request needs more than the whole arena  */
#define LBESSEL_ETIMEOUT (-5)   /* wait ended before the request was done   */
#define LBESSEL_ESTOPPED (-6)   /* the server is shutting down              */

#define LBESSEL_SERVE_BATCHED 0
#define LBESSEL_SERVE_PLAIN 1

typedef struct lbessel_server lbessel_server_t;

typedef struct lbessel_server_config {
    int64_t arena_bytes;        /* device arena for request data (> 0)           */
    int streams;                /* batches (plain: requests) in flight, 1..16   */
    int mode;                   /* LBESSEL_SERVE_BATCHED or LBESSEL_SERVE_PLAIN  */
    int max_batch_requests;     /* requests per batch, 1..1024                   */
    int64_t max_batch_elems;    /* evaluation pairs per batch (>= 1); a single
                                   larger request still forms a batch alone    */
    int poll_us;                /* scheduler sleep while batches run; 0 = spin  */
    int64_t solo_elems;         /* evaluation requests of at least this many
                                   pairs, and vMF fits, form a batch alone
                                   (>= 1)                                       */
} lbessel_server_config_t;

/* Request states in lbessel_request_info_t.state */
#define LBESSEL_REQ_QUEUED 0
#define LBESSEL_REQ_ADMITTED 1
#define LBESSEL_REQ_LAUNCHED 2
#define LBESSEL_REQ_DONE 3

/* Times are seconds on the server clock (lbessel_server_clock). */
typedef struct lbessel_request_info {
    int status;          /* LBESSEL_OK or the error that ended the request */
    int state;           /* LBESSEL_REQ_*                                 */
    int64_t batch;       /* sequence number of the batch that ran it      */
    int64_t bytes;       /* arena bytes it held                           */
    double t_arrival;    /* scheduled arrival (replay) or t_submit        */
    double t_submit;
    double t_admit;
    double t_launch;
    double t_done;
} lbessel_request_info_t;

typedef struct lbessel_server_stats {
    int64_t submitted;
    int64_t completed;
    int64_t batches;
    int64_t kernel_launches;    /* evaluation launches (segmented or plain)    */
    int64_t eval_pairs;         /* pairs of completed evaluation requests      */
    int64_t vmf_fits;
    int64_t arena_bytes;
    int64_t arena_peak_bytes;   /* most arena bytes held at once               */
    int64_t queue_peak;         /* most requests waiting for admission at once */
    int64_t max_batch_requests_seen;
} lbessel_server_stats_t;

/* Default configuration: 2 GiB arena, 8 streams, batched, 64 requests and
 * 2^18 pairs per batch, evaluation requests of 2^16 pairs or more and vMF
 * fits alone, spinning scheduler.  With host-resident requests the server is
 * bound by the copies: a large request gains nothing from sharing a launch
 * and would make its batch-mates wait for its inputs, so only the small
 * requests, for which a launch costs as much as their copies, share
 * segmented launches. */
void lbessel_server_default_config(lbessel_server_config_t *cfg);

/*
 * Create a server on the current HIP device.  Returns LBESSEL_OK and *out,
 * LBESSEL_EINVAL for a bad configuration, LBESSEL_ENODEV without a usable
 * device, LBESSEL_EHIP if an allocation or stream creation failed.
 */
int lbessel_server_create(const lbessel_server_config_t *cfg, lbessel_server_t **out);

/*
 * Queue an evaluation request.  v, x: host arrays of n elements (double for
 * precision 64, float for 32); out: host array of n elements receiving the
 * log-values.  n = 0 is a valid (empty) request.  *ticket identifies it.
 * Errors: LBESSEL_EINVAL (bad kind/precision, n < 0, NULL with n > 0),
 * LBESSEL_ETOOBIG, LBESSEL_ESTOPPED; nothing is queued on error.
 */
int lbessel_server_submit_eval(lbessel_server_t *s, int kind, int precision, const void *v,
                               const void *x, void *out, int64_t n, int64_t *ticket);

/*
 * Queue a device-resident evaluation request: v, x, out DEVICE arrays of n
 * elements (double for precision 64, float for 32), complete before the call
 * (the server's streams do not wait on the caller's); out receives the
 * log-values.  The request holds no arena memory.  Errors as for
 * lbessel_server_submit_eval.
 */
int lbessel_server_submit_eval_device(lbessel_server_t *s, int kind, int precision,
                                      const void *v, const void *x, void *out, int64_t n,
                                      int64_t *ticket);

/*
 * Queue a vMF fit: X device, row-major float32, n rows of p columns
 * (1 <= n <= 2^31 - 1, p >= 2), complete before the call (the server's
 * streams do not wait on the caller's); result: host, 4 doubles as in
 * lbessel_vmf_fit_f32.  Errors as for submit_eval.
 */
int lbessel_server_submit_vmf(lbessel_server_t *s, const float *X, int64_t n, int64_t p,
                              double *result, int64_t *ticket);

/*
 * Wait until the request is done or timeout_s seconds have passed
 * (timeout_s < 0: no limit).  Returns the request's status (LBESSEL_OK when
 * its outputs are in place) and releases the ticket, or LBESSEL_ETIMEOUT
 * (the ticket stays valid and the request still runs: its buffers must
 * stay valid until it is done or the server is destroyed), or
 * LBESSEL_EINVAL for an unknown ticket.
 * info (may be NULL) receives the request's record.
 */
int lbessel_server_wait(lbessel_server_t *s, int64_t ticket, double timeout_s,
                        lbessel_request_info_t *info);

/* Seconds since the server was created (steady clock). */
double lbessel_server_clock(lbessel_server_t *s);

int lbessel_server_stats(lbessel_server_t *s, lbessel_server_stats_t *st);

/* Finish all queued work, stop the scheduler, free the server. */
int lbessel_server_destroy(lbessel_server_t *s);

/*
 * Open-loop load replay: submit items[i] at t_arrival seconds after the
 * call starts (items sorted by t_arrival), from the calling thread, then
 * wait for all of them.  info[i] receives each record, with t_arrival the
 * scheduled time, so t_done - t_arrival is the latency a client sees.
 * type 0 = evaluation (kind, precision, v, x, out, n) with host arrays,
 * 1 = vMF fit (X, n, p, result), 2 = evaluation with device arrays
 * (lbessel_server_submit_eval_device); any other type is LBESSEL_EINVAL.
 * Returns LBESSEL_OK, or the first error (submission errors stop the replay;
 * requests already queued are still waited for).
 */
typedef struct lbessel_replay_item {
    double t_arrival;
    int type;
    int kind;
    int precision;
    int reserved;
    const void *v;
    const void *x;
    void *out;
    int64_t n;
    const float *X;
    int64_t p;
    double *result;
} lbessel_replay_item_t;

int lbessel_server_replay(lbessel_server_t *s, const lbessel_replay_item_t *items, int64_t count,
                          double timeout_s, lbessel_request_info_t *info);

#ifdef __cplusplus
}
#endif

#endif /* LBESSEL_SERVE_H */
