/*
 * pt_serve.h -- continuous-batching serving engine of libptmg.
 *
 * Requests are coupled pressure-temperature solves (the problem of
 * pt_mg.h: the implicit solve of Eqs. 27-28 that Algorithm 1 runs once per
 * time step) of any grid size.  The engine owns one device arena (the HBM
 * budget) and a fixed set of HIP streams ("slots").  A submitted request
 * queues; it is admitted, in arrival order, as soon as a slot is free and
 * its footprint (pt_mg_footprint_bytes plus its right-hand side) fits in
 * the free arena.  Its hierarchy is then assembled and solved on its own
 * stream, in steps that the engine enqueues as the previous ones finish,
 * so the work of all admitted requests overlaps on the device.  On
 * completion the arena block and the slot are released and waiting
 * requests are admitted.  Every request's kernels are the library's
 * deterministic ones on its own stream, so its result is the same bits
 * alone or in any mix.
 *
 * The engine is driven by its caller's thread through pt_server_progress
 * (no hidden threads).  No device or pinned memory is allocated after
 * pt_server_create.
 *
 * Conventions: as in pt_mg.h (device float64 arrays, x fastest).  The
 * arrays a request names (problem fields, right-hand side, outputs) must
 * stay valid until the request has finished.
 */
#ifndef PT_SERVE_H
#define PT_SERVE_H

#include <stddef.h>

#include "pt_mg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pt_server_s *pt_server_t;

typedef struct {
    size_t hbm_budget;   /* bytes of the device arena holding admitted requests */
    int max_active;      /* slots: requests on the device at once, 1..64 */
    int use_graphs;      /* replay each request's coarse-level cycle from a HIP graph */
    int omega_milli;     /* PT_OPT_OMEGA of every request's handle (0: the default) */
    int coarse_sweeps;   /* PT_OPT_COARSE_SWEEPS of every request's handle (0: the default) */
} pt_server_config;

/* Request states reported before the solve's own pt_status. */
#define PT_SERVE_QUEUED (-3)
#define PT_SERVE_ACTIVE (-2)

typedef struct {
    int status;            /* PT_SERVE_QUEUED, PT_SERVE_ACTIVE, or the final pt_status */
    int cycles;            /* V-cycles of the solve */
    double relres[2];      /* final (p, T) relative residual, paper row form */
    double t_arrival;      /* as given to pt_server_submit */
    double t_admit;        /* admission time (pt_server_now clock) */
    double t_done;         /* time the engine saw the result complete */
    size_t bytes;          /* arena bytes the request held */
} pt_request_info;

/* Seconds on the engine's monotonic clock. */
double pt_server_now(void);

/* Allocates the arena, pinned status memory and the slot streams (default
 * priority).  PT_ERR_ARG on a bad config, PT_ERR_OOM if the arena cannot be
 * allocated. */
int pt_server_create(const pt_server_config *cfg, pt_server_t *out);

/* Queue one request.  prob, precision: as pt_mg_setup.  b_p, b_T: the
 * mode-native right-hand side, or NULL in PT_COEF_PHASES mode to form the
 * paper's (Eqs. 33-34) from prob's p_adv/T_adv and div_ustar (NULL = 0)
 * inside the engine.  p, T: outputs [N] (zero initial guess unless
 * opts->zero_guess == 0, then also the guess).  opts NULL: pt_mg_solve's
 * defaults.  t_arrival: the request's arrival time on the pt_server_now
 * clock (latency is measured from it).  *id receives the request id.
 * PT_ERR_ARG for an invalid problem; a request larger than the whole
 * arena is accepted and finishes with PT_ERR_OOM. */
int pt_server_submit(pt_server_t s, const pt_problem *prob, int precision, const double *b_p,
                     const double *b_T, const double *div_ustar, double *p, double *T,
                     const pt_solve_opts *opts, double t_arrival, long long *id);

/* Run the engine loop (admit, poll, enqueue next steps) until the clock
 * reaches `until` (waiting when idle), or, with until = +infinity, until
 * nothing is queued or active.  *n_done (may be NULL) receives the number
 * of requests that finished during the call. */
int pt_server_progress(pt_server_t s, double until, int *n_done);

/* State and timings of one request (finished requests are kept). */
int pt_server_request(pt_server_t s, long long id, pt_request_info *info);

/* Counts: queued, active, finished requests, and arena bytes in use. */
int pt_server_stats(pt_server_t s, int *queued, int *active, long long *finished,
                    size_t *bytes_in_use);

/* Waits for the active requests, then frees everything. */
void pt_server_destroy(pt_server_t s);

const char *pt_server_last_error(pt_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* PT_SERVE_H */
