/*
 * lpk serving: many LPs solved together on one MI355X.
 *
 * Each LP is the problem statement of lpk.h (the paper's primal-dual pair) solved by the
 * same interior-point method.  A single LP of moderate size leaves most of the GPU idle
 * (every Krylov iteration is a short chain of dependent kernels), so throughput comes
 * from solving many at once in lockstep: the LPs of a batch run the same phase of their
 * own interior-point iteration together, and each phase is one kernel launch covering all
 * of them (one workgroup row per LP).  An LP that finishes leaves the batch at the end of
 * an iteration and a waiting one joins; it computes its starting point during the next
 * iteration.  Every reduction of an LP is partitioned by that LP's own sizes, so its
 * result is bitwise the same alone and in any batch.
 *
 * Conventions as in lpk.h: every call returns an lp_status, nothing aborts, host arrays
 * are copied at the call.
 */
#ifndef LPK_SERVER_H
#define LPK_SERVER_H

#include "lpk.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Solve `count` already-created problems, up to `width` of them in lockstep.  Problems
 * that share inner iterations, sweeps, Krylov method and layout (sparse / dense) form one
 * group (FP32 and FP64 sweeps share a group: each launch serves the members of its
 * precision); groups run one after the other, each on a stream of its own (every problem's
 * stream is synchronised first).  results[i] receives lp_solve's result for problems[i]
 * (seconds: from joining the batch to leaving it).  Returns LP_OK when every solve ran
 * (check results[i].status), else the first error.  Errors: LP_EINVAL (NULL arrays,
 * count < 0, width < 1), LP_EDEVICE.                                                      */
lp_status lp_solve_batch(lp_problem** problems, int32_t count, int32_t width, lp_result* results);

/* lp_time_kernel for a batch: the launches of kernel class cls for all `count` problems
 * together (one launch covers every problem), replayed `reps` times between two HIP
 * events.  bytes and flops are summed over the problems.  The problems must share inner
 * iterations, sweeps, Krylov method and layout, and each needs a scaling (a solve ran).
 * Errors: LP_EINVAL, LP_EDEVICE.                                                          */
lp_status lp_time_batch_kernel(lp_problem** problems, int32_t count, int32_t cls, int32_t reps,
                               double* us_per_launch, double* bytes_per_launch,
                               double* flops_per_launch, int32_t* launches_per_group);

typedef struct lp_server lp_server;

typedef struct {
    int32_t slots;           /* LPs solved at once, over all lanes, [1, 256] [32]           */
    int32_t max_skip;        /* FIFO with bounded skip: later requests that may start ahead
                                of a head request that does not fit yet [8]                */
    int32_t lanes;           /* lockstep batches the slots are split into, [1, 8] [1].  Each
                                lane runs on a stream of its own and the engine thread keeps
                                every lane's next round queued, so one lane's latency-bound
                                launches (a small LP's one-block sweep lasts as long as its
                                chain of colour steps) overlap another lane's bandwidth-bound
                                ones.  Every LP's arithmetic is the same in any lane.      */
    int32_t pad0;
    uint64_t hbm_budget;     /* device bytes the admitted problems may hold together, by
                                lp_footprint_bytes [0: 80% of the free memory at create]     */
    lp_options solver;       /* options for every request (device_io and stream ignored)    */
} lp_server_options;

typedef struct {
    uint64_t ticket;
    int32_t status;          /* lp_solve's status, or the lp_create error, or LP_ETOOBIG     */
    int32_t iters;           /* interior-point iterations                                  */
    double pobj, dobj, gamma_rel;
    int64_t krylov_iters;
    double t_submit, t_start, t_done;   /* seconds since lp_server_create                  */
    uint64_t footprint;      /* bytes charged against the budget                          */
} lp_completion;

lp_status lp_server_options_default(lp_server_options* o);

/* Start the server on the current HIP device: a preparer thread (admission, lp_create, and
 * lp_destroy of finished problems, whose device memory is released to the budget then) and
 * an engine thread that runs the lanes.  Errors: LP_EINVAL, LP_EDEVICE.                  */
lp_status lp_server_create(const lp_server_options* o, lp_server** out);

/* Queue one LP (host arrays, validated and copied now; same layout as lp_create).  A
 * request whose footprint exceeds the whole budget completes at once with LP_ETOOBIG.
 * Errors: those of lp_create's validation (the request is not queued then).             */
lp_status lp_server_submit(lp_server* s, int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                           const int32_t* col_idx, const double* val, const double* b,
                           const double* c, uint64_t* ticket);

/* Completions not yet returned (up to cap), without blocking.                           */
lp_status lp_server_poll(lp_server* s, lp_completion* out, int32_t cap, int32_t* n_out);

/* Block until at least `count` completions wait to be polled, or every submitted request
 * has completed, or timeout_s seconds pass (then LP_NOT_CONVERGED).                     */
lp_status lp_server_wait(lp_server* s, int32_t count, double timeout_s);

/* Copy a completed request's solution (x: n, y: m, s: n; any may be NULL) and release it.
 * Errors: LP_EINVAL (unknown ticket or not completed).                                  */
lp_status lp_server_result(lp_server* s, uint64_t ticket, double* x, double* y, double* s_out);

/* Device bytes currently held by admitted requests, and requests waiting in the queue.   */
lp_status lp_server_stats(lp_server* s, uint64_t* bytes_in_use, int32_t* queued, int32_t* running);

/* Finish the running and queued requests, stop the workers, free everything.            */
lp_status lp_server_destroy(lp_server* s);

#ifdef __cplusplus
}
#endif

#endif /* LPK_SERVER_H */
