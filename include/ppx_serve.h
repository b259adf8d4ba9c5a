/*
 * ppx_serve.h -- a continuous-batching request loop over the batched
 * operations of ppx.h.  Jobs (ppx_job: a whole batched FFT, scan or
 * tridiagonal call) arrive one by one; the server admits them in arrival
 * order while their memory fits an HBM budget, packs every job admitted
 * since its last launch into ONE mixed persistent launch (launch_mixed),
 * keeps up to `max_inflight` launches running on separate streams so that new
 * work overlaps work already on the device, retires jobs when their launch's
 * completion event fires, and returns their memory to the budget when the
 * client releases them.  The per-request mode launches every admitted job on
 * its own with the single call (fft_batched / scan_batched / tridiag_batched)
 * and is the baseline.
 *
 * The paper evaluates each operation as one batched call per problem set
 * (Sec. IV-A, Sec. VI); serving a stream of uneven requests this way is an
 * extension of that batched invocation, not a method of the paper.
 *
 * Memory: a job's footprint is its input plus output bytes; admission needs
 * footprint(admitted, unreleased) + footprint(job) <= budget.  A job whose
 * `out` is NULL gets its output allocated from a device arena of `budget`
 * bytes the server owns (first fit, 256-byte aligned), valid until released.
 * Times are host steady-clock microseconds since the server was created.
 * A server is not thread-safe: drive it from one thread.
 */
#ifndef PPX_SERVE_H
#define PPX_SERVE_H

#include <stdint.h>

#include "ppx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ppx_server ppx_server;

#define PPX_SERVE_FUSED 0        /* continuous batching into mixed launches */
#define PPX_SERVE_PER_REQUEST 1  /* one single-call launch per job (baseline) */
#define PPX_SERVE_NULL_DEVICE 2  /* OR-able: no GPU; launches complete at the
                                    next progress call (bookkeeping tests) */
#define PPX_SERVE_ONLINE_TUNE 4  /* OR-able with PPX_SERVE_PER_REQUEST: online
                                    learned tuning (ppx_online_* of
                                    ppx_tune.h) per (op, dtype, n, tridiagonal
                                    family); a job of >= 2^20 elements, when
                                    its class awaits no other cost, launches
                                    the session's next candidate and is timed
                                    with events (cost: ns per element); every
                                    other launch uses the class's current
                                    choice.  Results do not depend on the
                                    candidate beyond rounding. */

typedef struct ppx_completion {
    int64_t id;
    void *out;           /* the job's output (server arena or client buffer) */
    double arrival_us;   /* submit time, or the trace's arrival time in replay */
    double admit_us;     /* when it was admitted and launched */
    double complete_us;  /* when its launch's completion was observed */
} ppx_completion;

typedef struct ppx_server_stats {
    int64_t submitted, admitted, completed, released, launches;
    int64_t budget_bytes, used_bytes, peak_used_bytes;
    int32_t max_inflight_seen, pending;
} ppx_server_stats;

/* max_inflight: launches on the device at once (1..4). */
int ppx_server_create(int64_t hbm_budget_bytes, int max_inflight, int flags, ppx_server **out);
int ppx_server_destroy(ppx_server *s);

/* Queues a job (validated as launch_mixed would; out may be NULL).  Fails
 * with PPX_ENOMEM if the job alone exceeds the budget.  Never blocks. */
int ppx_server_submit(ppx_server *s, const ppx_job *job, int64_t *id);

/* Non-blocking step: retire finished launches, then admit and launch what
 * fits.  *launched (optional) receives the number of jobs launched. */
int ppx_server_progress(ppx_server *s, int *launched);

/* Moves up to cap completed jobs to out[]; *count receives how many. */
int ppx_server_poll(ppx_server *s, ppx_completion *out, int cap, int *count);

/* Returns a completed job's memory to the budget (and its output to the
 * arena when the server allocated it). */
int ppx_server_release(ppx_server *s, int64_t id);

/* Copies `bytes` of a completed, unreleased job's output to host memory. */
int ppx_server_read(ppx_server *s, int64_t id, void *host_dst, int64_t bytes);

int ppx_server_stats_get(ppx_server *s, ppx_server_stats *out);

/* Online tuning (PPX_SERVE_ONLINE_TUNE): sessions (job classes) seen,
 * evaluation launches so far, sessions whose search has stopped. */
int ppx_server_online_stats(ppx_server *s, int *sessions, int64_t *evaluations, int *converged);

/* A request of a replayed trace: the job and its arrival time (us after the
 * replay starts). */
typedef struct ppx_request {
    ppx_job job;
    double arrival_us;
} ppx_request;

/*
 * Replays a trace in real time: submits each request when the host clock
 * reaches its arrival time, drives progress/poll until every request has
 * completed, and writes completions in request order to out[n].  With
 * auto_release the server releases each job as soon as it completes.
 */
int ppx_serve_replay(ppx_server *s, const ppx_request *reqs, int n, int auto_release,
                     ppx_completion *out);

#ifdef __cplusplus
}
#endif

#endif /* PPX_SERVE_H */
