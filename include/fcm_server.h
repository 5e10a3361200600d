/*
 * fcm_server.h -- C ABI of the fast-FCM request server (continuous batching of
 * mobility evaluations on one GPU).
 *
 * Each request is one application of the fast-FCM mobility (Sec. 4 of Su &
 * Keaveny, arXiv 2310.12651) with its own particle count, box (cubic, or
 * rectangular through fcm_server_submit_box), kernel width, grid and cut-off.  A worker thread inside the library admits pending requests
 * whenever a slot is free and the device bytes of the plan the request needs fit
 * the server's budget, runs up to `slots` requests at once on separate
 * (non-blocking, default-priority) HIP streams so their kernels overlap on the
 * GPU, and retires them as their completion events fire.  Plans (grids,
 * twiddles, sort and cell-list buffers) stay resident and are re-bound to later
 * requests with the same grid, support and precision; idle plans are released,
 * least recently used first, when the budget needs room.
 *
 * Admission: requests are taken in arrival order, except that one waiting for
 * device memory held by running requests (or, with max_points, for grid points
 * in flight) may be passed by later requests that fit, at most 32 times; after
 * that nothing is admitted past it.  max_points bounds the grid work in flight,
 * so that a large request is not slowed by as many others as there are slots.
 *
 * Ownership and ordering: request arrays are caller-owned DEVICE pointers
 * (N x 3 FP64, as in fcm_mobility) that must stay valid, and must not be
 * written by the caller, until the request is done.  The request runs on the
 * server's own streams: inputs written by device work must either be complete
 * at submit, or be queued on the stream named in `after_stream`, which the
 * request then waits for.  Results land in V and Omega in the caller's order.
 * A request with a non-finite position completes with FCM_ENONFINITE (its
 * outputs are those of the position wrapped to 0, as in fcm_mobility).
 * Every call returns an FCM_* status (fcm.h); no exception crosses the ABI.
 */
#ifndef FCM_SERVER_H
#define FCM_SERVER_H

#include <stdint.h>

#include "fcm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FCM_EBUSY (-6) /* the pending queue is full: retry later */

typedef struct fcm_server_impl* fcm_server_t;

typedef struct {
    int64_t N;           /* particles                                        */
    double L;            /* periodic box side                                */
    double a;            /* particle radius                                  */
    double sigma_delta;  /* Sigma, modified kernel width (>= a / sqrt(pi))   */
    int grid;            /* grid points per axis (even 2^p 3^q, 8..1024)     */
    double r_cut;        /* pair-correction cut-off, 0 <= r_cut < L/2        */
    int support;         /* M_G, 0 = automatic (as fcm_options.support)      */
    double eta;          /* viscosity (0 = 1)                                */
    const double* pos;   /* device N x 3                                     */
    const double* F;     /* device N x 3                                     */
    const double* T;     /* device N x 3 or NULL (zero torques)              */
    double* V;           /* device N x 3, written                            */
    double* Omega;       /* device N x 3, written, or NULL                   */
    void* after_stream;  /* hipStream_t of the caller, or NULL: the request  */
                         /* runs after the work queued there before submit   */
                         /* (e.g. the kernels that wrote pos, F and T)       */
} fcm_request;

typedef struct {
    int64_t max_bytes;   /* device bytes for plans; 0 = 80 % of free memory  */
    int slots;           /* requests in flight at once (default 8, <= 64)    */
    int precision;       /* FCM_FP64 or FCM_FP32_BULK (default)              */
    int kahan;           /* as fcm_options.kahan (default 0)                 */
    int max_queue;       /* pending requests accepted (default 4096)         */
    int64_t max_points;  /* grid points of the requests in flight at most;   */
                         /* 0 = no limit (default); one request always runs  */
} fcm_server_options;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t plans_built, plans_rebound, plans_evicted;
    int64_t bytes_in_use, bytes_peak;
    int inflight_peak;
} fcm_server_stats;

/* Fill `opt` with the defaults above. */
int fcm_server_options_default(fcm_server_options* opt);
/* Start a server (worker thread) on the current HIP device. */
int fcm_server_create(fcm_server_t* out, const fcm_server_options* opt);
/* Queue a request; *ticket identifies it.  The parameters are validated here
 * (FCM_EINVAL / FCM_ERANGE as for fcm_plan); FCM_EBUSY if the queue is full. */
int fcm_server_submit(fcm_server_t s, const fcm_request* req, int64_t* ticket);
/* Queue a request on a rectangular periodic box, as fcm_plan_box: L (host, 3
 * sides along x, y, z) and grid (host, 3 point counts, one grid spacing on all
 * axes) replace the request's own L and grid fields, which are ignored; the
 * library copies both arrays.  The rod and filament runs of Sec. 6.3 use such
 * grids (512 x 512 x 8, 256 x 256 x 16).  A cached plan is re-bound only to a
 * request with the same three grid sizes.  Errors: as fcm_server_submit, and as
 * fcm_plan_box for the box (unequal spacings, a support longer than an axis it
 * may not wrap on); FCM_EINVAL if L or grid is NULL. */
int fcm_server_submit_box(fcm_server_t s, const fcm_request* req, const double L[3], const int grid[3],
                          int64_t* ticket);
/* *state = 0 queued, 1 running, 2 done; returns the request's status once done. */
int fcm_server_poll(fcm_server_t s, int64_t ticket, int* state);
/* Block until the request is done; queue_ms = submit -> launch, run_ms =
 * launch -> completion seen by the server (either may be NULL).  Returns the
 * request's status (FCM_ENOMEM if its plan can never fit the budget,
 * FCM_ENONFINITE for a non-finite position) and forgets the ticket.  One thread
 * may wait for a ticket: a second concurrent waiter gets FCM_EINVAL, as does a
 * ticket already waited for. */
int fcm_server_wait(fcm_server_t s, int64_t ticket, double* queue_ms, double* run_ms);
/* Counters since creation. */
int fcm_server_get_stats(fcm_server_t s, fcm_server_stats* out);
/* Finish all queued and running requests, release every plan, stop the worker. */
int fcm_server_destroy(fcm_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* FCM_SERVER_H */
