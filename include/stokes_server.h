/*
 * stokes_server.h -- a request server for permeability solves on one GPU
 * (continuous batching).  Not part of the paper's method: it serves many
 * independent solves of the problem that stokes.h states (Sec. 2), each
 * exactly as a context of its own would compute it: a one-member
 * stokes_setup_batch context for mixed-precision requests, stokes_setup_on_stream
 * for FP64 ones.
 *
 * Requests enter a FIFO queue.  `slots` host worker threads, each with its own
 * non-blocking HIP stream on the device current at stokes_server_create, take
 * the request at the head of the queue as soon as a slot is free and its
 * device bytes (stokes_estimate_bytes, FP32 vectors included when precision is
 * 1) fit in what the HBM budget has left.  A slot that takes a mixed-precision
 * request also takes, in queue order, the queued requests of the same box
 * size, force, preconditioner and tolerance whose bytes still fit the budget,
 * up to the batching caps (stokes_server_set_batching), and solves them on one
 * batched context: each kernel launch advances all of them.  Requests that
 * arrive while others run are admitted as slots and memory free up; their
 * kernels overlap on the device (set GPU_MAX_HW_QUEUES to at least `slots`
 * before the process first uses HIP for every slot to have its own hardware
 * queue).  A request's result is bitwise the same alone or among others.
 *
 * Thread safety: every call may be made from any thread, except that no call
 * may overlap or follow stokes_server_destroy on the same server.
 */
#ifndef STOKES_SERVER_H
#define STOKES_SERVER_H

#include "stokes.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stokes_server stokes_server;

typedef struct {
    int64_t id;
    int status;                 /* stokes_status of setup + solve (STOKES_E_STATE: cancelled) */
    int N;
    double k_hat;               /* permeability (stokes_report.k_hat) */
    int outer_iters, inner_A_iters, inner_S_iters;
    double rel_res;             /* ||g - S p|| / ||g|| at the end */
    double div_norm;            /* ||B u|| of the returned velocity */
    int64_t device_bytes;       /* bytes the request's context held */
    double t_submit;            /* server clock (seconds since create): queued */
    double t_start;             /* admitted to a slot */
    double t_end;               /* result ready */
    int batch_members;          /* requests that shared its context (1: alone) */
} stokes_request_result;

/* Start a server with `slots` workers (1..64) and an HBM budget in bytes
 * (> 0) for the contexts of running requests.  STOKES_E_DEVICE when no HIP
 * device is current. */
stokes_status stokes_server_create(stokes_server **srv, int slots, int64_t hbm_budget_bytes);

/* Queue one request.  mask: host pointer to N^3 bytes (copied during the
 * call), N, force: as for stokes_setup; precond, tol: as for stokes_solve;
 * precision: 0 FP64, 1 mixed (the "precision" option).  *id receives the
 * request id.  STOKES_E_ARG for bad arguments (the mask bytes are checked
 * when the request runs, and reported in its status), STOKES_E_LIMIT when the
 * request alone exceeds the budget, STOKES_E_STATE after destroy began. */
stokes_status stokes_server_submit(stokes_server *srv, const uint8_t *mask, int N, const double force[3],
                                   stokes_precond precond, double tol, int precision, int64_t *id);

/* Block until request `id` is done and copy its result (results stay
 * available until stokes_server_destroy).  STOKES_E_ARG for an unknown id. */
stokes_status stokes_server_wait(stokes_server *srv, int64_t id, stokes_request_result *result);

/* Batching caps: at most max_members (1..32; 1 = no batching) requests and
 * max_cells voxels (members x N^3) per batched context.  Defaults 32 and 2^21
 * (one 128^3 box: beyond that a context fills the GPU on its own).
 * STOKES_E_ARG for values out of range. */
stokes_status stokes_server_set_batching(stokes_server *srv, int max_members, int64_t max_cells);

/* stats[0..9]: submitted, completed, queued, running, bytes in use, peak
 * bytes in use, peak running requests, budget, contexts started (batches,
 * single requests included), requests run on them. */
stokes_status stokes_server_stats(stokes_server *srv, int64_t stats[10]);

/* Seconds since stokes_server_create on the server's clock (0 for NULL). */
double stokes_server_clock(stokes_server *srv);

/* Cancel queued requests, let running ones finish, join the workers and free
 * the server.  NULL is ignored. */
void stokes_server_destroy(stokes_server *srv);

#ifdef __cplusplus
}
#endif

#endif
