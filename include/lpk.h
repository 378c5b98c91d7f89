/*
 * lpk -- interior-point search directions for LP on AMD Instinct MI355X (gfx950).
 *
 * Problem (the primal-dual pair of the paper's introduction):
 *     min c^T x  s.t.  A x = b, x >= 0        max b^T y  s.t.  A^T y + s = c, s >= 0
 * with A an m x n matrix, m <= n, possibly rank deficient (duplicated rows are fine, no
 * presolve is needed: the min-norm formulation of Sec. 2.2 never breaks down).
 *
 * The method is Mehrotra's predictor-corrector interior-point algorithm (Sec. 2.1) whose
 * search directions come from the min-norm problem  min ||dw|| s.t. (A D) dw = f
 * (Sec. 2.2, eq. minnrmprob; D = S^-1/2 X^1/2), row-scaled so that every row of
 * A_hat = diag(rho)^-1 A D has unit norm (Sec. 3.5), and solved by AB-GMRES
 * right-preconditioned by inner iterations (Sec. 3.2, 3.4): multicolour NE-SOR sweeps,
 * NE-SSOR sweeps, Cimmino sweeps, or (for dense A) SOR on the explicit Gram matrix
 * A_hat A_hat^T; or by CGNE or MRNE preconditioned by the same sparse inner iterations
 * (Sec. 3.3); or by BA-GMRES, GMRES on the left-preconditioned normal equations of the
 * first kind C A_hat A_hat^T dyh = C f_hat in m-space (the corrector-stage remark of
 * Sec. 3.2, eq. ba_ne), C the NE-SOR or NE-SSOR operator, with dw = A_hat^T dyh.
 * The direction is recovered with the w-recurrence (eq. step_predictor /
 * step_corrector), saving one matrix-vector product per stage.
 *
 * Conventions for every entry point:
 *  - every call returns an lp_status; LP_OK == 0.  No exception or abort crosses the ABI.
 *    lp_last_error() returns a thread-local message describing the last failure.
 *  - A is 0-based CSR: row_ptr[m+1] (int64, row_ptr[0] == 0, non-decreasing),
 *    col_idx[nnz] (int32, strictly increasing inside each row, 0 <= j < n), val[nnz].
 *  - vectors are contiguous double arrays; m-vectors are in the caller's row order.
 *  - when lp_options.device_io == 1 every caller array (inputs and outputs) is a device
 *    pointer on the current HIP device (e.g. a torch tensor's data_ptr()); otherwise a
 *    host pointer.  Inputs are copied at the call; the caller keeps ownership of all of
 *    its arrays and may free them after the call returns.
 *  - all device work is ordered on lp_options.stream (a hipStream_t; NULL = the legacy
 *    default stream).  Calls return after their results are in the caller's arrays.
 *  - an lp_problem is used by one thread at a time.
 */
#ifndef LPK_H
#define LPK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LP_OK = 0,
    LP_EINVAL = 1,          /* malformed input (CSR structure, empty row or column, NULL) */
    LP_EDIM = 2,            /* dimensions: m > n, m < 1, sizes beyond 2^31 - 1 entries    */
    LP_ENONFINITE = 3,      /* NaN or Inf in A, b, c or a vector argument                 */
    LP_ENOMEM = 4,          /* device or host allocation failed                           */
    LP_ETOOBIG = 5,         /* request exceeds a fixed limit or budget                    */
    LP_EDEVICE = 6,         /* no usable HIP device, or a HIP call failed                 */
    LP_NOT_CONVERGED = 7,   /* iteration limit reached (Sec. 4.2: 99 iterations)          */
    LP_DIVERGED = 8,        /* iterate became non-finite or non-positive                  */
    LP_KRYLOV_MAXIT = 9     /* reserved: Krylov limit is reported in lp_krylov_info       */
} lp_status;

/* LP_MIXED: FP32 inner sweeps (and their products) with the outer Krylov method, the true
 * residual and the interior-point update in FP64, where FP32 pays: NE-SOR / NE-SSOR sweeps
 * stay in FP64 when an LP's sweep runs in one workgroup from LDS in FP64 (z, v_k, p_k and
 * the row pointers, and the rows if they fit, in the 160 KiB of LDS; the LP then computes
 * as with LP_FP64), and run in FP32 otherwise (FP32 halves z, which may then fit in LDS,
 * and the bytes streamed from memory).  Cimmino and the dense path run in FP32.  LPs whose
 * sweeps run in different precisions share batches.                                    */
typedef enum { LP_FP64 = 0, LP_MIXED = 1 } lp_precision;
typedef enum { LP_ABGMRES = 0, LP_CGNE = 1, LP_MRNE = 2, LP_BAGMRES = 3 } lp_krylov;
typedef enum { LP_NESOR = 0, LP_CIMMINO = 1, LP_NESSOR = 2, LP_GSOR = 3 } lp_inner;

typedef struct lp_problem lp_problem;

/* Options.  lp_options_default() fills the values given in brackets. */
typedef struct {
    int32_t precision;       /* lp_precision [LP_FP64]                                    */
    int32_t krylov;          /* lp_krylov [LP_ABGMRES]; LP_CGNE / LP_MRNE run the sweeps   */
                             /* of LP_NESOR, LP_NESSOR or LP_CIMMINO on the sparse rows    */
                             /* (with lp_create_dense: LP_NESSOR or LP_CIMMINO); LP_MRNE   */
                             /* needs precision LP_FP64; LP_BAGMRES needs lp_create,      */
                             /* LP_NESOR or LP_NESSOR and precision LP_FP64; it stops on  */
                             /* its own residual |gamma_k| <= tol ||C f_hat||, and         */
                             /* lp_krylov_info.res_est is that residual                   */
    int32_t inner;           /* lp_inner [LP_NESOR]; LP_GSOR needs lp_create_dense        */
    int32_t inner_sweeps;    /* ell, inner iterations per preconditioner application [2]; */
                             /* an NE-SSOR iteration is a forward and a backward sweep     */
    double omega;            /* NE-SOR relaxation, (0, 2) [1.0]                           */
    double omega_c;          /* Cimmino step; <= 0: 1/lambda, lambda from 20 power steps [0] */
    int64_t krylov_max_iter; /* Krylov iteration limit; <= 0 means m (Sec. 4.2) [0]       */
    int32_t ipm_max_iter;    /* interior-point iteration limit [99] (Sec. 4.2)            */
    int32_t start;           /* 0: Mehrotra starting point; 1: lp_set_state's point [0]   */
    double eps_out;          /* stopping tolerance on gamma_rel [1e-8]                    */
    double eta;              /* step-length damping in [0.9, 1) [0.9995] (eq. steplength) */
    double phi;              /* centrality parameter [1e-5] (Sec. 2.1)                    */
    double sigma_max;        /* sigma cap [0.208] (Sec. 2.1)                              */
    double eps_in0;          /* first Krylov tolerance [1e-6] (Sec. 4.2)                  */
    double eps_in_min;       /* [1e-14]                                                   */
    double eps_in_max;       /* [1e-4]                                                    */
    double init_tol;         /* Krylov tolerance of the two starting-point solves [1e-10] */
    double backtrack;        /* back-tracking factor for the centrality test [0.95]       */
    int32_t max_backtrack;   /* [200]                                                     */
    int32_t device_io;       /* 1: caller arrays are device pointers [0]                  */
    void* stream;            /* hipStream_t [NULL]                                        */
    int32_t poll_every;      /* Krylov iterations enqueued between convergence checks [0=auto] */
    int32_t use_graphs;      /* 1: replay each Krylov iteration as a captured HIP graph [1] */
    int32_t schedule;        /* batches (lp_solve_batch, lp_server): 0 auto = members of one */
                             /* structure (equal m, n, nnz) pass each phase together, others */
                             /* advance alone; 1 always together; 2 always alone [0]; a     */
                             /* member asking 2 wins over 1, 1 over 0                       */
    int32_t max_correctors;  /* multiple centrality correctors per step, in [0, 8] [0]:    */
                             /* 0 is Mehrotra's predictor-corrector step of Sec. 2.1; K > 0 */
                             /* adds up to K correctors of Gondzio's multi-corrector method */
                             /* (the framework the paper names as future work), each one   */
                             /* more min-norm solve of the corrector's form (eq.            */
                             /* step_corrector with target products): aim at step lengths  */
                             /* 0.1 longer, move the products at that trial point into     */
                             /* [0.1, 10] sigma mu (decreases capped at 10 sigma mu), keep  */
                             /* the corrected direction if its shorter step length grows by */
                             /* at least 0.01; stop at the first miss                       */
} lp_options;

/* Per direction solve (Sec. 4.2 stopping rule ||f_hat - A_hat dw|| <= eps_in ||f_hat||). */
typedef struct {
    int64_t iters;           /* Krylov iterations                                         */
    double beta;             /* ||f_hat||                                                  */
    double res_est;          /* residual of the stopping test for the returned iterate:   */
                             /* AB-GMRES the Givens estimate |gamma_{k+1}|, BA-GMRES its  */
                             /* preconditioned residual, CGNE / MRNE ||f_hat - A_hat dw|| */
                             /* recomputed from dw                                        */
    double res_true;         /* ||f_hat - A_hat dw||, recomputed at exit                  */
    int32_t failed;          /* 1: tolerance not met within the limit (Sec. 4.2 rule)     */
    int32_t pad0;
} lp_krylov_info;

/* Per interior-point iteration; the measures describe the iterate at the step's entry. */
typedef struct {
    double mu;               /* x^T s / n                                                  */
    double gamma;            /* error measure, eq. errorMeasureDef                         */
    double gamma_rel;        /* same with |c^T x - b^T y| / max(1, |c^T x|) in place of mu */
    double rp_rel, rd_rel, gap_rel, pobj, dobj;
    double alpha_p, alpha_d, sigma, eps_in;
    double res_af, res_cc;   /* relative true residuals of the two solves                 */
    int64_t k_af, k_cc;      /* Krylov iterations of the two solves                       */
    int32_t fail_af, fail_cc, backtracks;
    int32_t converged;       /* 1: the stopping test held at entry; no step was taken     */
    int32_t correctors;      /* centrality correctors accepted (lp_options.max_correctors) */
    int32_t pad0;
    int64_t k_mcc;           /* Krylov iterations of the centrality correctors' solves     */
} lp_iter_info;

/* Interior-point state beyond (x, y, s): enough to resume at an iteration boundary.     */
typedef struct {
    double eps_in;           /* current Krylov tolerance                                   */
    int32_t k;               /* interior-point iterations taken                           */
    int32_t fail_prev;       /* 1: a solve of the previous iteration failed (Sec. 4.2)    */
} lp_ipm_state;

typedef struct {
    int32_t status;          /* LP_OK, LP_NOT_CONVERGED or LP_DIVERGED                    */
    int32_t iters;           /* interior-point iterations                                  */
    double gamma, gamma_rel, pobj, dobj, rp_rel, rd_rel, gap_rel;
    int64_t krylov_iters;    /* total Krylov iterations over the solve                    */
    double seconds;          /* wall time of lp_solve                                      */
} lp_result;

/* Fill o with the defaults listed above.  Errors: LP_EINVAL if o is NULL.               */
lp_status lp_options_default(lp_options* o);

/* Problem statement (introduction, eq. PrimalDualPair).  Validates A, b, c on the host
 * (host inputs) before any device call, copies them to the device, builds the greedy
 * row colouring (rows sharing no column share a colour; colour-major order is the
 * NE-SOR sweep order), the CSC copy of A and all solver workspace.  Errors: LP_EINVAL
 * (NULL pointers, malformed CSR, empty row or column), LP_EDIM (m < 1, m > n, nnz or
 * sizes >= 2^31), LP_ENONFINITE, LP_ENOMEM, LP_EDEVICE.  *out is NULL on error.      */
lp_status lp_create(int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                    const int32_t* col_idx, const double* val, const double* b, const double* c,
                    const lp_options* o, lp_problem** out);

/* Same problem with A dense, row-major with leading dimension lda >= n.  The inner
 * iterations default to SOR on the explicit Gram matrix G = A_hat A_hat^T formed once per
 * interior-point step with FP64 matrix cores (equal in exact arithmetic to NE-SOR in
 * natural row order, Sec. 3.4).  Zero entries are kept.  Errors as lp_create.          */
lp_status lp_create_dense(int64_t m, int64_t n, const double* A, int64_t lda, const double* b,
                          const double* c, const lp_options* o, lp_problem** out);

/* The same problem with general bounds: min c^T x s.t. A x = b, lo <= x <= hi, with
 * lo[j] = -INFINITY and hi[j] = +INFINITY allowed (n each; host or device per
 * device_io, like the other inputs).  As for the typical LPs of the experiments
 * (Sec. 4.3, after LIPSOL), the problem is brought to the standard form of the
 * introduction on the host and that form is solved:
 *   lo finite, hi infinite:  x_j = lo_j + x'_j
 *   both finite, lo < hi:    x_j = lo_j + x'_j plus a row x'_j + w_j = hi_j - lo_j, w_j >= 0
 *   lo infinite, hi finite:  x_j = hi_j - x'_j
 *   both infinite (free):    x_j = x+_j - x-_j
 *   lo == hi (fixed):        x_j = lo_j, the column leaves the problem.
 * Standard-form columns: the kept variables in order, then the negative parts of the
 * free variables, then the slacks; rows: the rows of A, then one row per boxed variable
 * (lp_bounds_standard_form returns exactly this form).  Every other entry point then
 * works on the standard form (lp_get_state returns its x, y, s; lp_result's objectives
 * omit the constant sum_j c_j shift_j); lp_bounded_solution maps the iterate back.
 * m > n is allowed when the standard form has m' <= n'.
 * Errors: those of lp_create; LP_EINVAL also for NaN bounds, lo_j = +inf, hi_j = -inf,
 * lo_j > hi_j, or a row whose variables are all fixed; LP_EDIM when m' > n'.            */
lp_status lp_create_bounded(int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                            const int32_t* col_idx, const double* val, const double* b, const double* c,
                            const double* lo, const double* hi, const lp_options* o, lp_problem** out);

/* For a problem made by lp_create_bounded: the current iterate in the caller's
 * variables, x[n] (lo <= x <= hi up to the iterate's interiority), the multipliers y[m]
 * of the rows of A (the first m of the standard form's, caller's row order), and
 * *obj = c^T x.  x, y host or device per device_io (either may be NULL); obj a host
 * pointer (may be NULL).  Errors: LP_EINVAL (NULL p, or p not made by lp_create_bounded),
 * LP_EDEVICE.                                                                          */
lp_status lp_bounded_solution(const lp_problem* p, double* x, double* y, double* obj);

/* The standard form of lp_create_bounded on the host alone (no device needed; host
 * arrays).  First call with row_ptr_out == NULL: sizes only (*m_out, *n_out, *nnz_out).
 * Second call with caller-allocated row_ptr_out[m'+1], col_idx_out[nnz'], val_out[nnz'],
 * b_out[m'], c_out[n'] and optionally offset (the objective constant).
 * Errors: LP_EINVAL (malformed CSR, invalid bounds, a row of fixed variables, NULL),
 * LP_ENONFINITE (b, c or A), LP_EDIM.                                                   */
lp_status lp_bounds_standard_form(int64_t m, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                                  const double* val, const double* b, const double* c, const double* lo,
                                  const double* hi, int64_t* m_out, int64_t* n_out, int64_t* nnz_out,
                                  int64_t* row_ptr_out, int32_t* col_idx_out, double* val_out, double* b_out,
                                  double* c_out, double* offset);

/* Release every device and host resource of p (NULL is a no-op).                        */
void lp_destroy(lp_problem* p);

/* One iteration of Mehrotra's predictor-corrector algorithm (Sec. 2.1) from the current
 * iterate: residuals and the error measure, eps_in schedule (Sec. 4.2), D-scaling and
 * row scaling (Sec. 2.2, 3.5), predictor solve and w-recurrence (eq. step_predictor),
 * step lengths (eq. steplength), sigma rule, corrector solve (eq. step_corrector),
 * centrality back-tracking, update.  If the stopping test gamma_rel <= eps_out holds at
 * entry, info->converged = 1 and nothing changes.  The first call on a new problem
 * computes the starting point first (unless options.start == 1).
 * Errors: LP_DIVERGED (non-finite or non-positive iterate), LP_EDEVICE.               */
lp_status ipm_step(lp_problem* p, lp_iter_info* info);

/* The search-direction solve (Sec. 2.2, eq. minnrmprob) on its own:
 *     min ||dw||  s.t.  (A diag(d)) dw = f,     dw = (A diag(d))^T dy,
 * solved on the row-scaled system (Sec. 3.5) by the configured Krylov method and inner
 * iterations from dw_0 = 0, stopping when ||f_hat - A_hat dw|| <= tol ||f_hat||.
 * d: n positive entries, or NULL for the current D = sqrt(x/s); f: m entries (R(A D)).
 * dw: n outputs; dy: m outputs or NULL.  ki may be NULL.  Krylov non-convergence is not
 * an error: ki->failed = 1 and, as Sec. 4.2 prescribes for a solve that misses its
 * tolerance, the iterate of least residual norm is returned.  For AB-GMRES and BA-GMRES
 * that is the last iterate (their minimised residual does not grow); CGNE and MRNE, whose
 * residual may grow, test ||f_hat - A_hat dw|| recomputed after every step and keep the
 * least-residual iterate seen (dw_0 = 0 included).
 * Errors: LP_EINVAL (NULL f or dw, tol < 0), LP_ENONFINITE, LP_EDEVICE.                */
lp_status direction_solve(lp_problem* p, const double* d, const double* f, double tol,
                          double* dw, double* dy, lp_krylov_info* ki);

/* For callers that cannot allocate device memory during the call (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): direction_solve with
 * every per-call device buffer -- the batch descriptors, the Krylov control block, the
 * phase parameters, the reduction partials and the Krylov workspace (basis V, multiplier
 * vectors P, Hessenberg matrix, Givens and Gram-Schmidt arrays) -- in one fixed device array
 * of 32 MiB that the library holds on each GPU it runs on until the process ends.  The
 * call allocates nothing (no hipMalloc, hipFree, pinned host allocation or graph
 * instantiation) and launches the kernels of direction_solve one by one, so its results
 * are those of direction_solve.  d (n doubles, or NULL for the current D), f (m), dw (n)
 * and dy (m, or NULL) are device pointers on the current device whatever
 * lp_options.device_io says; the problem must have been created on this device.  The
 * array is shared by every call on a GPU and keeps the last call's contents (each call
 * sets up what it reads): calls that overlap on one GPU, from other threads or on other
 * streams, race and must be serialised by the caller.
 * Errors: those of direction_solve; LP_ETOOBIG when the workspace (for AB-GMRES about
 * 16 m (kmax + 1) + 8 (kmax + 1)^2 bytes) exceeds the array (create the problem with a
 * smaller krylov_max_iter); LP_EDEVICE when the current device is not the problem's.   */
lp_status direction_solve_noalloc(lp_problem* p, const double* d, const double* f, double tol,
                                  double* dw, double* dy, lp_krylov_info* ki);

/* The whole interior-point solve: starting point (unless options.start == 1), then
 * ipm_step until gamma_rel <= eps_out or ipm_max_iter iterations (Sec. 4.2).  Returns the
 * final status (LP_OK, LP_NOT_CONVERGED, LP_DIVERGED or an error); r may be NULL.       */
lp_status lp_solve(lp_problem* p, lp_result* r);

/* Copy the current iterate out (x: n, y: m, s: n; any may be NULL) and, if st is not
 * NULL, the interior-point state.                                                      */
lp_status lp_get_state(const lp_problem* p, double* x, double* y, double* s, lp_ipm_state* st);

/* Replace the iterate and state (resume, or start from a given point with start == 1).
 * x and s must be positive.  st may be NULL (eps_in = eps_in0, k = 0, fail_prev = 0).
 * Errors: LP_EINVAL (NULL x/y/s, non-positive x or s), LP_ENONFINITE.                  */
lp_status lp_set_state(lp_problem* p, const double* x, const double* y, const double* s,
                       const lp_ipm_state* st);

/* Per-iteration log of the last lp_solve: up to cap entries into info, count in *n_out. */
lp_status lp_get_log(const lp_problem* p, lp_iter_info* info, int32_t cap, int32_t* n_out);

/* Device bytes lp_create would allocate for an m x n problem with nnz nonzeros and the
 * given options (NULL = defaults), including (AB-GMRES, BA-GMRES) the Krylov basis of
 * krylov_max_iter + 1 vectors (AB-GMRES also keeps as many multiplier vectors); CGNE
 * and MRNE keep a fixed number of vectors.  Where NE-SOR / NE-SSOR sweeps colour by
 * colour, the count includes the largest possible row slices (a second copy of at most
 * 5/4 nnz elements that lp_create builds only for colours whose rows touch neighbouring
 * columns), so it is an upper bound there.
 * Errors: LP_EDIM.                                                                    */
lp_status lp_footprint_bytes(int64_t m, int64_t n, int64_t nnz, const lp_options* o,
                             uint64_t* bytes);

/* How the inner-iteration sweeps of p run (either pointer may be NULL): *fp32 = 1 when
 * they run in FP32 (LP_MIXED where it pays, see lp_precision), and for NE-SOR / NE-SSOR on
 * sparse rows *kind = 2 when each preconditioner application runs in one workgroup with
 * the rows, z, v_k and p_k in LDS, 1 when z, v_k and p_k are in LDS and the rows are read
 * from memory, 0 when the sweeps run colour by colour over many workgroups (and for the
 * other inner iterations).  Host only.  Errors: LP_EINVAL (NULL p).                    */
lp_status lp_sweep_layout(const lp_problem* p, int32_t* fp32, int32_t* kind);

/* Number of colours of the row colouring and the colour sizes (sizes may be NULL).      */
lp_status lp_colouring(const lp_problem* p, int32_t* ncolours, int32_t* sizes, int32_t cap);

/* Presolve of dependent rows (the preprocessing the conclusions name), host only: rows
 * of A that are scalar multiples of an earlier row, exact duplicates included.  Row k is
 * such a multiple of row i when both have the same columns and a_kj / a_k0 equals
 * a_ij / a_i0 to tol (relative; tol = 0 asks for equality), lambda = a_k0 / a_i0.
 * keep[m] receives 0 for those rows and 1 for the others, *m_keep the rows kept; the
 * caller builds the reduced LP from the kept rows (the duals of the dropped rows may be
 * taken as 0).  Dependencies among three or more rows are left in place here (the
 * min-norm formulation of Sec. 2.2 solves rank-deficient problems as they are); the
 * general search is lp_presolve_dependent_rows.
 * Errors: LP_EINVAL (malformed CSR, NULL, tol < 0, or a dropped row whose right-hand
 * side is not lambda times its partner's to tol: the LP is infeasible),
 * LP_ENONFINITE, LP_EDIM.                                                              */
lp_status lp_presolve_rows(int64_t m, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                           const double* val, const double* b, double tol, int32_t* keep, int64_t* m_keep);

/* Presolve of general dependent rows (the conclusions' "detect and remove linear
 * dependencies"), host only: keep[k] = 0 exactly when row k of A is in the span of rows
 * 0..k-1, so the kept rows are the first row basis in the given order and number rank(A);
 * *m_keep receives that count.  Found by sparse elimination, one row at a time: a row is
 * dependent when its remainder after elimination against the kept rows is at most tol times
 * its largest entry (relative; 1e-9 suits data of moderate condition).  Its right-hand side,
 * eliminated alongside, must vanish to tol relative to the terms that formed it, else the LP
 * is infeasible.  Rows that are multiples of another (lp_presolve_rows) are among those
 * found; so is the transportation matrix's single dependency (one of its rows).  The caller
 * builds the reduced LP from the kept rows; the dropped rows' duals may be taken as 0.
 * Errors: LP_EINVAL (malformed CSR, NULL, tol < 0, contradicting right-hand side),
 * LP_ENONFINITE, LP_EDIM, LP_ETOOBIG (the elimination would store more than
 * max(32 nnz, 4M) entries), LP_ENOMEM.                                                  */
lp_status lp_presolve_dependent_rows(int64_t m, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                                     const double* val, const double* b, double tol, int32_t* keep,
                                     int64_t* m_keep);

/* Greedy row colouring on the host alone (no device needed): colour[m] and the
 * colour-major sweep order perm[m] (rows ascending inside each colour).
 * Errors: LP_EINVAL (malformed CSR).                                                   */
lp_status lp_colour_rows(int64_t m, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                         int32_t* colour, int32_t* perm, int32_t* ncolours);

/* Kernel classes timed by the profiler.                                                */
typedef enum {
    LP_K_SWEEP = 0,          /* one colour of a NE-SOR sweep, or one Cimmino half-sweep     */
    LP_K_SPMV_CSR = 1,       /* u = A_hat z of the Krylov loop (FP64)                       */
    LP_K_SPMV_CSC = 2,       /* z = A_hat^T p of the Krylov loop (FP64)                     */
    LP_K_GS_DOTS = 3,        /* Gram-Schmidt dot products V^T u                             */
    LP_K_GS_UPDATE = 4,      /* Gram-Schmidt update u -= V h (with the next dots or norm)   */
    LP_K_GRAM = 5,           /* dense path: G = A_hat A_hat^T with FP64 matrix cores        */
    LP_K_CG_VEC = 6,         /* CGNE / MRNE dot products and vector updates                 */
    LP_K_COUNT = 7
} lp_kernel_class;

typedef struct {
    int32_t cls;             /* lp_kernel_class                                            */
    int32_t pad0;
    int64_t launches;        /* launches that did work (skipped launches are not counted)  */
    double ms_total;         /* sum of HIP-event durations of those launches              */
    double bytes_total;      /* algorithmic bytes: each input and output moved once       */
    double flops_total;      /* algorithmic floating-point operations                     */
    char name[32];
} lp_kernel_stat;

/* Per-launch HIP-event timing, on the problem's stream, of the kernel classes whose bit
 * (1 << class) is set in mask (0 turns profiling off and clears the statistics).
 * Timing adds two event records per launch; use it outside throughput measurements.   */
lp_status lp_profile(lp_problem* p, uint32_t mask);

/* Accumulated statistics since lp_profile was called: one entry per class (up to cap
 * entries into st; the count in *n_out).  Synchronises the stream.                    */
lp_status lp_profile_read(lp_problem* p, lp_kernel_stat* st, int32_t cap, int32_t* n_out);

/* Mean duration of one launch of kernel class cls (LP_K_SWEEP: one application of the
 * inner-iteration preconditioner; LP_K_SPMV_CSR / LP_K_SPMV_CSC: the Krylov loop's two
 * products; LP_K_GS_DOTS / LP_K_GS_UPDATE: the AB- or BA-GMRES Gram-Schmidt passes at basis
 * size min(128, krylov limit); LP_K_GRAM: the dense path's Gram and preconditioner
 * build, timed per launch of its kernels), from `reps` back-to-back replays of its
 * launches captured with the current A_hat, between two HIP events on the problem's
 * stream.  Also returns the algorithmic bytes and flops per launch (as in
 * lp_kernel_stat) and the launches in one group (e.g. colours x sweeps).  Needs a
 * scaling: run ipm_step, lp_solve or direction_solve first.  Overwrites the Krylov
 * workspace (column 0, and for the Gram-Schmidt classes one column of H and u).
 * Errors: LP_EINVAL, LP_EDEVICE.                                                        */
lp_status lp_time_kernel(lp_problem* p, int32_t cls, int32_t reps, double* us_per_launch,
                         double* bytes_per_launch, double* flops_per_launch,
                         int32_t* launches_per_group);

/* Human-readable name of a status code (static storage).                               */
const char* lp_status_str(lp_status s);

/* Thread-local description of the last error returned on this thread ("" if none).     */
const char* lp_last_error(void);

/* Library version string.                                                              */
const char* lp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LPK_H */
