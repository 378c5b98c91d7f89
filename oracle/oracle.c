/*
 * CPU FP64 ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded implementation of the interior-point search-direction
 * path of Cui, Morikuni, Tsuchiya and Hayami, "Implementation of interior-point methods
 * for LP based on Krylov subspace iterative solvers with inner-iteration
 * preconditioning".  It exists only to check the GPU library: only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * helper or table with the GPU library.
 *
 * Conventions: all arithmetic in IEEE double, built with -ffp-contract=off (no fused
 * multiply-add) and without fast-math; every dot product and norm is summed in index
 * order.  A is 0-based CSR with sorted unique column indices per row.
 *
 * Function map (section / equation / algorithm of the paper each one follows):
 *   orc_colour            greedy row colouring; gives the row order of the NE-SOR sweep
 *                         (the paper sweeps rows 1..m; any fixed order is an SOR sweep)
 *   orc_nesor             NE-SOR inner iterations, Algorithm "NE-SOR method" (Sec. 3.4)
 *   orc_nessor            NE-SSOR inner iterations, Algorithm "NE-SSOR method" (Sec. 3.3)
 *   orc_cimmino           Cimmino inner iterations (not in the paper; the simultaneous
 *                         counterpart of NE-SOR on the same normal equations)
 *   orc_scale             D-scaling A -> AD (Sec. 2.2) and row scaling by the row norms of
 *                         AD (Sec. 3.5, eq. scaleD / scaled_ls)
 *   orc_dirsolve          min-norm problem (eq. minnrmprob) by AB-GMRES (Algorithm
 *                         "AB-GMRES method preconditioned by inner iterations", Sec. 3.2),
 *                         CGNE or MRNE (Algorithms of Sec. 3.1) on the row-scaled system,
 *                         or BA-GMRES (the corrector-stage remark of Sec. 3.2, eq. ba_ne)
 *   orc_affine_direction  predictor stage via the w-recurrence (eq. step_predictor)
 *   orc_corrector_direction corrector stage via the w-recurrence (eq. step_corrector)
 *   orc_init_point        starting point (Mehrotra's published heuristic; the paper
 *                         defers to LIPSOL, whose code is not reproduced here)
 *   orc_ipm_iterate       one iteration of Mehrotra's predictor-corrector algorithm
 *                         (Sec. 2.1, eq. steplength, the sigma rule, eq. errorMeasureDef,
 *                         the centrality back-tracking, the eps_in schedule of Sec. 4.2)
 *   orc_ipm               the whole interior-point loop (Sec. 4.2 limits)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ----------------------------------------------------------------------------------- */
/* status codes of the oracle                                                           */
enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOMEM = 4, ORC_NOT_CONVERGED = 7, ORC_DIVERGED = 8 };

/* inner iteration kinds, Krylov kinds, sweep orders */
enum { ORC_NESOR = 0, ORC_CIMMINO = 1, ORC_NESSOR = 2 };
enum { ORC_ABGMRES = 0, ORC_CGNE = 1, ORC_MRNE = 2, ORC_BAGMRES = 3 };
enum { ORC_ORDER_COLOUR = 0, ORC_ORDER_NATURAL = 1 };

typedef struct {
    int32_t krylov;     /* ORC_ABGMRES / ORC_CGNE / ORC_MRNE / ORC_BAGMRES */
    int32_t inner;      /* ORC_NESOR / ORC_CIMMINO / ORC_NESSOR */
    int32_t ell;        /* inner sweeps per preconditioner application */
    int32_t order;      /* ORC_ORDER_COLOUR or ORC_ORDER_NATURAL */
    int32_t flexible;   /* AB-GMRES final step: 0 = apply B to V y, 1 = A^T (P y) */
    int32_t pad0;
    double omega;       /* relaxation parameter (NE-SOR / NE-SSOR) */
    double omega_c;     /* Cimmino step; <= 0 means 1/lambda from power iteration */
    int64_t kmax;       /* maximum Krylov iterations; <= 0 means m */
} orc_solver_opts;

typedef struct {
    int64_t iters;      /* Krylov iterations taken */
    double beta;        /* ||f_hat|| */
    double res_est;     /* residual the method reports (GMRES: |gamma_{k+1}|) */
    double res_true;    /* ||f_hat - A_hat dw|| recomputed at exit */
    int32_t failed;     /* 1: tolerance not reached within kmax */
    int32_t pad0;
    double omega_c;     /* Cimmino step actually used */
} orc_krylov_info;

typedef struct {
    orc_solver_opts solver;
    int32_t max_iter;   /* 99 */
    int32_t start;      /* 0: heuristic starting point; 1: caller's x, y, s */
    double eps_out;     /* 1e-8, applied to gamma_rel */
    double eta;         /* 0.9995 */
    double phi;         /* 1e-5 */
    double sigma_max;   /* 0.208 */
    double eps_in0, eps_in_min, eps_in_max;   /* 1e-6, 1e-14, 1e-4 */
    double init_tol;    /* tolerance of the two starting-point solves, 1e-10 */
    double backtrack;   /* 0.95 */
    int32_t max_backtrack; /* 200 */
    int32_t max_correctors; /* centrality correctors per step (0: Mehrotra's method alone) */
} orc_ipm_opts;

typedef struct {
    double mu, gamma, gamma_rel, rp_rel, rd_rel, gap_rel, pobj, dobj;
    double alpha_p, alpha_d, sigma, eps_in, res_af, res_cc;
    int64_t k_af, k_cc;
    int32_t fail_af, fail_cc, backtracks, correctors;   /* correctors accepted */
} orc_iter_log;

/* ----------------------------------------------------------------------------------- */
/* small dense helpers (index-order sums)                                               */
static double dot(int64_t n, const double* a, const double* b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}
static double nrm2(int64_t n, const double* a) { return sqrt(dot(n, a, a)); }

/* y = A x (CSR) */
static void csr_mv(int64_t m, const int64_t* rp, const int32_t* ci, const double* val,
                   const double* x, double* y) {
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += val[k] * x[ci[k]];
        y[i] = s;
    }
}
/* y = A^T x (CSR, scatter in row order) */
static void csr_tmv(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                    const double* x, double* y) {
    for (int64_t j = 0; j < n; ++j) y[j] = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) y[ci[k]] += val[k] * x[i];
}

/* exported so that tests can check the generators' products independently */
void orc_csr_mv(int64_t m, const int64_t* rp, const int32_t* ci, const double* val,
                const double* x, double* y) { csr_mv(m, rp, ci, val, x, y); }
void orc_csr_tmv(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                 const double* x, double* y) { csr_tmv(m, n, rp, ci, val, x, y); }

/* ----------------------------------------------------------------------------------- */
/* Greedy row colouring.  Row i gets the smallest colour not used by any earlier row    */
/* i' < i that has a nonzero in a common column.  Rows of one colour share no column,   */
/* so the NE-SOR updates of one colour touch disjoint entries of z.  The sweep order    */
/* is colour-major, rows ascending inside a colour.                                     */
int orc_colour(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci,
               int32_t* colour, int32_t* perm, int32_t* ncolours_out) {
    /* column lists (CSC pattern), rows ascending */
    int64_t* cp = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t nnz = rp[m];
    int32_t* ri = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    int64_t* fill = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* stamp = (int64_t*)malloc((size_t)(m + 1) * sizeof(int64_t));
    if (!cp || !ri || !fill || !stamp) { free(cp); free(ri); free(fill); free(stamp); return ORC_ENOMEM; }
    for (int64_t k = 0; k < nnz; ++k) cp[ci[k] + 1]++;
    for (int64_t j = 0; j < n; ++j) cp[j + 1] += cp[j];
    for (int64_t j = 0; j < n; ++j) fill[j] = cp[j];
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) ri[fill[ci[k]]++] = (int32_t)i;
    for (int64_t c = 0; c <= m; ++c) stamp[c] = -1;
    int32_t ncol = 0;
    for (int64_t i = 0; i < m; ++i) {
        /* mark the colours of earlier rows sharing a column with row i */
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t j = ci[k];
            for (int64_t t = cp[j]; t < cp[j + 1] && ri[t] < i; ++t) stamp[colour[ri[t]]] = i;
        }
        int32_t c = 0;
        while (stamp[c] == i) ++c;
        colour[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    /* colour-major order, ascending row index inside each colour (counting sort) */
    int64_t* start = (int64_t*)calloc((size_t)ncol + 1, sizeof(int64_t));
    if (!start) { free(cp); free(ri); free(fill); free(stamp); return ORC_ENOMEM; }
    for (int64_t i = 0; i < m; ++i) start[colour[i] + 1]++;
    for (int32_t c = 0; c < ncol; ++c) start[c + 1] += start[c];
    for (int64_t i = 0; i < m; ++i) perm[start[colour[i]]++] = (int32_t)i;
    *ncolours_out = ncol;
    free(start); free(cp); free(ri); free(fill); free(stamp);
    return ORC_OK;
}

/* the row order of one sweep */
static int make_order(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, int32_t order,
                      int32_t* perm) {
    if (order == ORC_ORDER_NATURAL) {
        for (int64_t i = 0; i < m; ++i) perm[i] = (int32_t)i;
        return ORC_OK;
    }
    int32_t* colour = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t nc = 0;
    if (!colour) return ORC_ENOMEM;
    int rc = orc_colour(m, n, rp, ci, colour, perm, &nc);
    free(colour);
    return rc;
}

/* ----------------------------------------------------------------------------------- */
/* NE-SOR inner iterations on  A A^T p = g,  z = A^T p  (Algorithm "NE-SOR method").     */
/* Starting from z = 0, p = 0, ell sweeps over the rows in the order perm:              */
/*   d_i = omega (g_i - alpha_i . z) / ||alpha_i||^2 ;  z += d_i alpha_i ;  p_i += d_i   */
/* rn2 holds ||alpha_i||^2; NULL means every row has unit norm (the row-scaled matrix   */
/* of Sec. 3.5, where the division is dropped).  p accumulates the multipliers, so that */
/* z = A^T p holds in exact arithmetic.                                                 */
void orc_nesor(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
               const double* rn2, const double* g, double omega, int32_t ell,
               const int32_t* perm, double* z, double* p) {
    for (int64_t j = 0; j < n; ++j) z[j] = 0.0;
    for (int64_t i = 0; i < m; ++i) p[i] = 0.0;
    for (int32_t sweep = 0; sweep < ell; ++sweep) {
        for (int64_t t = 0; t < m; ++t) {
            int64_t i = perm ? perm[t] : t;
            double s = 0.0;
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += val[k] * z[ci[k]];
            double d = omega * (g[i] - s);
            if (rn2) d = d / rn2[i];
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) z[ci[k]] += d * val[k];
            p[i] += d;
        }
    }
}

/* NE-SSOR inner iterations (Algorithm "NE-SSOR method"): each of the ell iterations is */
/* a forward sweep in the order perm followed by a backward sweep in the reverse order. */
void orc_nessor(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                const double* rn2, const double* g, double omega, int32_t ell,
                const int32_t* perm, double* z, double* p) {
    for (int64_t j = 0; j < n; ++j) z[j] = 0.0;
    for (int64_t i = 0; i < m; ++i) p[i] = 0.0;
    for (int32_t it = 0; it < ell; ++it) {
        for (int32_t dir = 0; dir < 2; ++dir) {
            for (int64_t t0 = 0; t0 < m; ++t0) {
                int64_t t = dir == 0 ? t0 : m - 1 - t0;
                int64_t i = perm ? perm[t] : t;
                double s = 0.0;
                for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += val[k] * z[ci[k]];
                double d = omega * (g[i] - s);
                if (rn2) d = d / rn2[i];
                for (int64_t k = rp[i]; k < rp[i + 1]; ++k) z[ci[k]] += d * val[k];
                p[i] += d;
            }
        }
    }
}

/* Cimmino inner iterations on the same normal equations: all rows at once,            */
/*   r = g - A z ;  p += omega_c r ;  z += omega_c A^T r   (ell times, from z = p = 0).  */
void orc_cimmino(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                 const double* g, double omega_c, int32_t ell, double* z, double* p) {
    double* r = (double*)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    double* t = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t j = 0; j < n; ++j) z[j] = 0.0;
    for (int64_t i = 0; i < m; ++i) p[i] = 0.0;
    for (int32_t it = 0; it < ell; ++it) {
        csr_mv(m, rp, ci, val, z, r);
        for (int64_t i = 0; i < m; ++i) r[i] = g[i] - r[i];
        for (int64_t i = 0; i < m; ++i) p[i] += omega_c * r[i];
        csr_tmv(m, n, rp, ci, val, r, t);
        for (int64_t j = 0; j < n; ++j) z[j] += omega_c * t[j];
    }
    free(r); free(t);
}

/* lambda estimate of A A^T: 20 power iterations from e/sqrt(m), lambda = ||A A^T v||    */
double orc_power_lambda(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci,
                        const double* val, int32_t iters) {
    double* v = (double*)malloc((size_t)m * sizeof(double));
    double* w = (double*)malloc((size_t)m * sizeof(double));
    double* t = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double lam = 0.0;
    for (int64_t i = 0; i < m; ++i) v[i] = 1.0 / sqrt((double)m);
    for (int32_t it = 0; it < iters; ++it) {
        csr_tmv(m, n, rp, ci, val, v, t);
        csr_mv(m, rp, ci, val, t, w);
        lam = nrm2(m, w);
        if (lam == 0.0) break;
        for (int64_t i = 0; i < m; ++i) v[i] = w[i] / lam;
    }
    free(v); free(w); free(t);
    return lam;
}

/* ----------------------------------------------------------------------------------- */
/* Scaling (Sec. 2.2 and Sec. 3.5): cal_A = A D with D = diag(d); rho_i = ||row i of     */
/* cal_A||_2; A_hat = diag(rho)^-1 cal_A.  The pattern of A_hat is that of A.             */
int orc_scale(int64_t m, const int64_t* rp, const int32_t* ci, const double* val, const double* d,
              double* rho, double* ahat) {
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            double a = val[k] * (d ? d[ci[k]] : 1.0);
            s += a * a;
        }
        rho[i] = sqrt(s);
        if (!(rho[i] > 0.0)) return ORC_EINVAL;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            ahat[k] = val[k] * (d ? d[ci[k]] : 1.0) / rho[i];
    }
    return ORC_OK;
}

/* one application of the inner-iteration preconditioner: (z, p) from g                */
static void apply_inner(const orc_solver_opts* o, int64_t m, int64_t n, const int64_t* rp,
                        const int32_t* ci, const double* ah, const int32_t* perm, double omega_c,
                        const double* g, double* z, double* p) {
    if (o->inner == ORC_CIMMINO)
        orc_cimmino(m, n, rp, ci, ah, g, omega_c, o->ell, z, p);
    else if (o->inner == ORC_NESSOR)
        orc_nessor(m, n, rp, ci, ah, NULL, g, o->omega, o->ell, perm, z, p);
    else
        orc_nesor(m, n, rp, ci, ah, NULL, g, o->omega, o->ell, perm, z, p);
}

/* AB-GMRES preconditioned by inner iterations, applied to A_hat dw = f_hat with         */
/* dw_0 = 0.  Arnoldi by modified Gram-Schmidt; the least-squares problem with the     */
/* Hessenberg matrix is solved by Givens rotations; the loop stops when the residual    */
/* |gamma_{k+1}| <= eps ||f_hat|| (the scaled-residual criterion of Sec. 4.2), when    */
/* h_{k+1,k} = 0, or at kmax.  Final step: literal (B applied to q_k = V_k y_k) or      */
/* flexible (dw = A_hat^T P y_k with the stored multiplier vectors P).  dyhat is the    */
/* multiplier vector with dw = A_hat^T dyhat.                                           */
static int abgmres(const orc_solver_opts* o, int64_t m, int64_t n, const int64_t* rp,
                   const int32_t* ci, const double* ah, const int32_t* perm, double omega_c,
                   const double* fh, double eps, int64_t kmax, double* dw, double* dyh,
                   orc_krylov_info* info) {
    double beta = nrm2(m, fh);
    info->beta = beta;
    info->iters = 0;
    info->res_est = beta;
    info->failed = 0;
    if (beta == 0.0) {
        memset(dw, 0, (size_t)n * sizeof(double));
        memset(dyh, 0, (size_t)m * sizeof(double));
        return ORC_OK;
    }
    int64_t ldh = kmax + 1;
    double* V = (double*)malloc((size_t)m * (size_t)(kmax + 1) * sizeof(double));
    double* P = o->flexible ? (double*)malloc((size_t)m * (size_t)kmax * sizeof(double)) : NULL;
    double* H = (double*)calloc((size_t)ldh * (size_t)kmax, sizeof(double));
    double* cs = (double*)malloc((size_t)kmax * sizeof(double));
    double* sn = (double*)malloc((size_t)kmax * sizeof(double));
    double* gam = (double*)calloc((size_t)kmax + 1, sizeof(double));
    double* z = (double*)malloc((size_t)n * sizeof(double));
    double* p = (double*)malloc((size_t)m * sizeof(double));
    double* u = (double*)malloc((size_t)m * sizeof(double));
    double* y = (double*)malloc((size_t)(kmax > 0 ? kmax : 1) * sizeof(double));
    if (!V || (o->flexible && !P) || !H || !cs || !sn || !gam || !z || !p || !u || !y) {
        free(V); free(P); free(H); free(cs); free(sn); free(gam); free(z); free(p); free(u); free(y);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < m; ++i) V[i] = fh[i] / beta;
    gam[0] = beta;
    int64_t k = 0;
    double res = beta;
    while (k < kmax) {
        double* vk = V + (size_t)k * m;
        apply_inner(o, m, n, rp, ci, ah, perm, omega_c, vk, z, p);
        if (P) memcpy(P + (size_t)k * m, p, (size_t)m * sizeof(double));
        csr_mv(m, rp, ci, ah, z, u);
        double* hk = H + (size_t)k * ldh;
        for (int64_t i = 0; i <= k; ++i) {
            double* vi = V + (size_t)i * m;
            hk[i] = dot(m, u, vi);
            for (int64_t t = 0; t < m; ++t) u[t] -= hk[i] * vi[t];
        }
        double hnext = nrm2(m, u);
        hk[k + 1] = hnext;
        if (hnext != 0.0) {
            double* vn = V + (size_t)(k + 1) * m;
            for (int64_t t = 0; t < m; ++t) vn[t] = u[t] / hnext;
        }
        /* previous rotations on the new column, then the rotation that zeroes h_{k+1,k} */
        for (int64_t i = 0; i < k; ++i) {
            double a = hk[i], b = hk[i + 1];
            hk[i] = cs[i] * a + sn[i] * b;
            hk[i + 1] = -sn[i] * a + cs[i] * b;
        }
        double a = hk[k], b = hk[k + 1];
        double r = hypot(a, b);
        if (r == 0.0) break;                /* singular column: keep the first k columns */
        cs[k] = a / r;
        sn[k] = b / r;
        hk[k] = r;
        hk[k + 1] = 0.0;
        gam[k + 1] = -sn[k] * gam[k];
        gam[k] = cs[k] * gam[k];
        res = fabs(gam[k + 1]);
        ++k;
        if (res <= eps * beta || hnext == 0.0) break;
    }
    /* back substitution R y = gamma(1:k) */
    for (int64_t i = k - 1; i >= 0; --i) {
        double s = gam[i];
        for (int64_t j = i + 1; j < k; ++j) s -= H[(size_t)j * ldh + i] * y[j];
        y[i] = s / H[(size_t)i * ldh + i];
    }
    if (o->flexible) {
        for (int64_t t = 0; t < m; ++t) {
            double s = 0.0;
            for (int64_t j = 0; j < k; ++j) s += P[(size_t)j * m + t] * y[j];
            dyh[t] = s;
        }
        csr_tmv(m, n, rp, ci, ah, dyh, dw);
    } else {
        for (int64_t t = 0; t < m; ++t) {
            double s = 0.0;
            for (int64_t j = 0; j < k; ++j) s += V[(size_t)j * m + t] * y[j];
            u[t] = s;
        }
        apply_inner(o, m, n, rp, ci, ah, perm, omega_c, u, dw, dyh);
    }
    info->iters = k;
    info->res_est = res;
    info->failed = (res > eps * beta) ? 1 : 0;
    free(V); free(P); free(H); free(cs); free(sn); free(gam); free(z); free(p); free(u); free(y);
    return ORC_OK;
}

/* The residual of the stopping rule of Sec. 4.2, ||f_hat - A_hat dw||, recomputed from dw  */
/* (CGNE and MRNE also carry a recurrence for it, which drifts from this value in        */
/* rounding; the stated criterion is on the residual itself).                           */
static double true_residual(int64_t m, const int64_t* rp, const int32_t* ci, const double* ah,
                            const double* fh, const double* dw, double* r) {
    csr_mv(m, rp, ci, ah, dw, r);
    for (int64_t i = 0; i < m; ++i) r[i] = fh[i] - r[i];
    return nrm2(m, r);
}

/* Sec. 4.2: a solve that fails to meet its tolerance adopts the iterate with the least   */
/* residual norm.  best_* hold that iterate (the initial dw_0 = 0 included); at the end, */
/* if the tolerance was missed and an earlier iterate had a smaller residual, it         */
/* replaces the last one.                                                                */
static void keep_least_residual(int64_t m, int64_t n, double res, double* best_res,
                                const double* dw, const double* dyh, double* bdw, double* bdyh) {
    if (res < *best_res) {
        *best_res = res;
        memcpy(bdw, dw, (size_t)n * sizeof(double));
        memcpy(bdyh, dyh, (size_t)m * sizeof(double));
    }
}

/* CGNE preconditioned by inner iterations (Algorithm "CGNE method preconditioned by    */
/* inner iterations"), dw_0 = 0, read with alpha_k in the update of dw.  The multiplier */
/* vector dyh is carried along (dyh += alpha_k * multipliers of q_k) so that             */
/* dw = A_hat^T dyh.  Stops when ||f_hat - A_hat dw_k|| <= eps ||f_hat|| or at kmax;     */
/* when the tolerance is missed the least-residual iterate is returned (Sec. 4.2).      */
static int cgne(const orc_solver_opts* o, int64_t m, int64_t n, const int64_t* rp,
                const int32_t* ci, const double* ah, const int32_t* perm, double omega_c,
                const double* fh, double eps, int64_t kmax, double* dw, double* dyh,
                orc_krylov_info* info) {
    double beta = nrm2(m, fh);
    info->beta = beta; info->iters = 0; info->res_est = beta; info->failed = 0;
    memset(dw, 0, (size_t)n * sizeof(double));
    memset(dyh, 0, (size_t)m * sizeof(double));
    if (beta == 0.0) return ORC_OK;
    double* g = (double*)malloc((size_t)m * sizeof(double));
    double* zz = (double*)malloc((size_t)m * sizeof(double));   /* z_k = C g_k (m-space) */
    double* uu = (double*)malloc((size_t)n * sizeof(double));   /* u_k = A^T z_k */
    double* q = (double*)malloc((size_t)n * sizeof(double));
    double* qm = (double*)malloc((size_t)m * sizeof(double));   /* multipliers of q */
    double* aq = (double*)malloc((size_t)m * sizeof(double));
    double* rt = (double*)malloc((size_t)m * sizeof(double));
    double* bdw = (double*)calloc((size_t)n, sizeof(double));
    double* bdyh = (double*)calloc((size_t)m, sizeof(double));
    memcpy(g, fh, (size_t)m * sizeof(double));
    apply_inner(o, m, n, rp, ci, ah, perm, omega_c, g, uu, zz);
    memcpy(q, uu, (size_t)n * sizeof(double));
    memcpy(qm, zz, (size_t)m * sizeof(double));
    double gamma = dot(m, g, zz);
    double res = beta, best = beta;
    int64_t k = 0;
    while (k < kmax) {
        double qq = dot(n, q, q);
        if (qq == 0.0) break;
        double alpha = gamma / qq;
        for (int64_t j = 0; j < n; ++j) dw[j] += alpha * q[j];
        for (int64_t i = 0; i < m; ++i) dyh[i] += alpha * qm[i];
        csr_mv(m, rp, ci, ah, q, aq);
        for (int64_t i = 0; i < m; ++i) g[i] -= alpha * aq[i];
        ++k;
        res = true_residual(m, rp, ci, ah, fh, dw, rt);
        if (res <= eps * beta) break;
        keep_least_residual(m, n, res, &best, dw, dyh, bdw, bdyh);
        apply_inner(o, m, n, rp, ci, ah, perm, omega_c, g, uu, zz);
        double gnew = dot(m, g, zz);
        double bk = gnew / gamma;
        gamma = gnew;
        for (int64_t j = 0; j < n; ++j) q[j] = uu[j] + bk * q[j];
        for (int64_t i = 0; i < m; ++i) qm[i] = zz[i] + bk * qm[i];
    }
    info->iters = k; info->failed = res > eps * beta;
    if (info->failed && best < res) {
        memcpy(dw, bdw, (size_t)n * sizeof(double));
        memcpy(dyh, bdyh, (size_t)m * sizeof(double));
        res = best;
    }
    info->res_est = res;
    free(g); free(zz); free(uu); free(q); free(qm); free(aq); free(rt); free(bdw); free(bdyh);
    return ORC_OK;
}

/* MRNE preconditioned by inner iterations (Algorithm "MRNE method preconditioned by    */
/* inner iterations"), read with consistent indices: dw_{k+1} = dw_k + alpha_k p_k,     */
/* gamma_{k+1} = ||q_{k+1}||^2, p_{k+1} = q_{k+1} + beta_k p_k.  Multipliers of p and q */
/* are carried so that dw = A_hat^T dyh.  Stops when ||f_hat - A_hat dw_k|| <=          */
/* eps ||f_hat|| or at kmax; when the tolerance is missed the least-residual iterate is */
/* returned (Sec. 4.2).                                                                 */
static int mrne(const orc_solver_opts* o, int64_t m, int64_t n, const int64_t* rp,
                const int32_t* ci, const double* ah, const int32_t* perm, double omega_c,
                const double* fh, double eps, int64_t kmax, double* dw, double* dyh,
                orc_krylov_info* info) {
    double beta = nrm2(m, fh);
    info->beta = beta; info->iters = 0; info->res_est = beta; info->failed = 0;
    memset(dw, 0, (size_t)n * sizeof(double));
    memset(dyh, 0, (size_t)m * sizeof(double));
    if (beta == 0.0) return ORC_OK;
    double* g = (double*)malloc((size_t)m * sizeof(double));
    double* q = (double*)malloc((size_t)n * sizeof(double));
    double* qm = (double*)malloc((size_t)m * sizeof(double));
    double* pv = (double*)malloc((size_t)n * sizeof(double));
    double* pm = (double*)malloc((size_t)m * sizeof(double));
    double* t = (double*)malloc((size_t)m * sizeof(double));
    double* v = (double*)malloc((size_t)n * sizeof(double));
    double* vm = (double*)malloc((size_t)m * sizeof(double));
    double* rt = (double*)malloc((size_t)m * sizeof(double));
    double* bdw = (double*)calloc((size_t)n, sizeof(double));
    double* bdyh = (double*)calloc((size_t)m, sizeof(double));
    memcpy(g, fh, (size_t)m * sizeof(double));
    apply_inner(o, m, n, rp, ci, ah, perm, omega_c, g, q, qm);   /* q_0 = A^T C g_0 */
    memcpy(pv, q, (size_t)n * sizeof(double));
    memcpy(pm, qm, (size_t)m * sizeof(double));
    double gamma = dot(n, q, q);
    double res = beta, best = beta;
    int64_t k = 0;
    while (k < kmax && gamma > 0.0) {
        csr_mv(m, rp, ci, ah, pv, t);                                /* t_k = A p_k */
        apply_inner(o, m, n, rp, ci, ah, perm, omega_c, t, v, vm);   /* v_k = A^T C t_k */
        double vp = dot(n, v, pv);
        if (vp == 0.0) break;
        double alpha = gamma / vp;
        for (int64_t j = 0; j < n; ++j) dw[j] += alpha * pv[j];
        for (int64_t i = 0; i < m; ++i) dyh[i] += alpha * pm[i];
        for (int64_t i = 0; i < m; ++i) g[i] -= alpha * t[i];
        for (int64_t j = 0; j < n; ++j) q[j] -= alpha * v[j];
        for (int64_t i = 0; i < m; ++i) qm[i] -= alpha * vm[i];
        ++k;
        res = true_residual(m, rp, ci, ah, fh, dw, rt);
        if (res <= eps * beta) break;
        keep_least_residual(m, n, res, &best, dw, dyh, bdw, bdyh);
        double gnew = dot(n, q, q);
        double bk = gnew / gamma;
        gamma = gnew;
        for (int64_t j = 0; j < n; ++j) pv[j] = q[j] + bk * pv[j];
        for (int64_t i = 0; i < m; ++i) pm[i] = qm[i] + bk * pm[i];
    }
    info->iters = k; info->failed = res > eps * beta;
    if (info->failed && best < res) {
        memcpy(dw, bdw, (size_t)n * sizeof(double));
        memcpy(dyh, bdyh, (size_t)m * sizeof(double));
        res = best;
    }
    info->res_est = res;
    free(g); free(q); free(qm); free(pv); free(pm); free(t); free(v); free(vm); free(rt);
    free(bdw); free(bdyh);
    return ORC_OK;
}

/* BA-GMRES (Hayami, Yin and Ito; the corrector-stage remark of Sec. 3.2) for the least-   */
/* squares form min ||A_hat^T dyh - h|| (eq. ba_ne) with the left preconditioner B = C A_hat */
/* of inner iterations: GMRES on B A_hat^T dyh = B h in m-space.  Here the right-hand side  */
/* is given as f_hat; when f_hat = A_hat h (the corrector) the Krylov space                 */
/* K(C A_hat A_hat^T, C f_hat) and the minimised norm ||C (f_hat - A_hat A_hat^T dyh)|| are  */
/* those of eq. ba_ne, and the same iteration applies to any f_hat in R(A_hat).  dyh_0 = 0; */
/* Arnoldi by MGS, the least-squares problem by Givens rotations; stop when the             */
/* preconditioned residual |gamma_{k+1}| <= eps ||C f_hat||, when h_{k+1,k} = 0 or at kmax. */
/* dw = A_hat^T dyh.                                                                         */
static int bagmres(const orc_solver_opts* o, int64_t m, int64_t n, const int64_t* rp,
                   const int32_t* ci, const double* ah, const int32_t* perm, double omega_c,
                   const double* fh, double eps, int64_t kmax, double* dw, double* dyh,
                   orc_krylov_info* info) {
    const double beta_f = nrm2(m, fh);
    info->beta = beta_f;
    info->iters = 0;
    info->res_est = 0.0;
    info->failed = 0;
    memset(dw, 0, (size_t)n * sizeof(double));
    memset(dyh, 0, (size_t)m * sizeof(double));
    if (beta_f == 0.0) return ORC_OK;
    int64_t ldh = kmax + 1;
    double* V = (double*)malloc((size_t)m * (size_t)(kmax + 1) * sizeof(double));
    double* H = (double*)calloc((size_t)ldh * (size_t)kmax, sizeof(double));
    double* cs = (double*)malloc((size_t)kmax * sizeof(double));
    double* sn = (double*)malloc((size_t)kmax * sizeof(double));
    double* gam = (double*)calloc((size_t)kmax + 1, sizeof(double));
    double* z = (double*)malloc((size_t)n * sizeof(double));
    double* t = (double*)malloc((size_t)n * sizeof(double));
    double* s = (double*)malloc((size_t)m * sizeof(double));
    double* u = (double*)malloc((size_t)m * sizeof(double));
    double* y = (double*)malloc((size_t)(kmax > 0 ? kmax : 1) * sizeof(double));
    if (!V || !H || !cs || !sn || !gam || !z || !t || !s || !u || !y) {
        free(V); free(H); free(cs); free(sn); free(gam); free(z); free(t); free(s); free(u); free(y);
        return ORC_ENOMEM;
    }
    /* r_0 = B h = C f_hat */
    apply_inner(o, m, n, rp, ci, ah, perm, omega_c, fh, z, u);
    const double beta = nrm2(m, u);
    info->res_est = beta;
    int64_t k = 0;
    double res = beta;
    if (beta > 0.0) {
        for (int64_t i = 0; i < m; ++i) V[i] = u[i] / beta;
        gam[0] = beta;
        while (k < kmax) {
            const double* vk = V + (size_t)k * m;
            csr_tmv(m, n, rp, ci, ah, vk, t);                        /* A_hat^T v_k */
            csr_mv(m, rp, ci, ah, t, s);                             /* A_hat A_hat^T v_k */
            apply_inner(o, m, n, rp, ci, ah, perm, omega_c, s, z, u); /* u = C s */
            double* hk = H + (size_t)k * ldh;
            for (int64_t i = 0; i <= k; ++i) {
                const double* vi = V + (size_t)i * m;
                hk[i] = dot(m, u, vi);
                for (int64_t r = 0; r < m; ++r) u[r] -= hk[i] * vi[r];
            }
            const double hnext = nrm2(m, u);
            hk[k + 1] = hnext;
            if (hnext != 0.0) {
                double* vn = V + (size_t)(k + 1) * m;
                for (int64_t r = 0; r < m; ++r) vn[r] = u[r] / hnext;
            }
            for (int64_t i = 0; i < k; ++i) {
                const double a = hk[i], b = hk[i + 1];
                hk[i] = cs[i] * a + sn[i] * b;
                hk[i + 1] = -sn[i] * a + cs[i] * b;
            }
            const double a = hk[k], b = hk[k + 1];
            const double r = hypot(a, b);
            if (r == 0.0) break;
            cs[k] = a / r;
            sn[k] = b / r;
            hk[k] = r;
            hk[k + 1] = 0.0;
            gam[k + 1] = -sn[k] * gam[k];
            gam[k] = cs[k] * gam[k];
            res = fabs(gam[k + 1]);
            ++k;
            if (res <= eps * beta || hnext == 0.0) break;
        }
        for (int64_t i = k - 1; i >= 0; --i) {
            double sum = gam[i];
            for (int64_t j = i + 1; j < k; ++j) sum -= H[(size_t)j * ldh + i] * y[j];
            y[i] = sum / H[(size_t)i * ldh + i];
        }
        for (int64_t r = 0; r < m; ++r) {
            double sum = 0.0;
            for (int64_t j = 0; j < k; ++j) sum += V[(size_t)j * m + r] * y[j];
            dyh[r] = sum;
        }
        csr_tmv(m, n, rp, ci, ah, dyh, dw);
    }
    info->iters = k;
    info->res_est = res;
    info->failed = res > eps * beta;
    free(V); free(H); free(cs); free(sn); free(gam); free(z); free(t); free(s); free(u); free(y);
    return ORC_OK;
}

/* ----------------------------------------------------------------------------------- */
/* The search-direction solve: min ||dw|| s.t. (A D) dw = f (eq. minnrmprob), solved on   */
/* the row-scaled system (eq. scaled_ls).  d may be NULL (D = I).  Outputs dw (n) and   */
/* dy (m) with dw = (A D)^T dy; dy = dyhat / rho.                                        */
int orc_dirsolve(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                 const double* d, const double* f, double eps, const orc_solver_opts* o,
                 double* dw, double* dy, orc_krylov_info* info) {
    int64_t nnz = rp[m];
    double* rho = (double*)malloc((size_t)m * sizeof(double));
    double* ah = (double*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    double* fh = (double*)malloc((size_t)m * sizeof(double));
    double* dyh = (double*)malloc((size_t)m * sizeof(double));
    double* r = (double*)malloc((size_t)m * sizeof(double));
    int32_t* perm = (int32_t*)malloc((size_t)m * sizeof(int32_t));
    int rc = ORC_ENOMEM;
    memset(info, 0, sizeof(*info));
    if (!rho || !ah || !fh || !dyh || !r || !perm) goto done;
    rc = orc_scale(m, rp, ci, val, d, rho, ah);
    if (rc != ORC_OK) goto done;
    for (int64_t i = 0; i < m; ++i) fh[i] = f[i] / rho[i];
    rc = make_order(m, n, rp, ci, o->order, perm);
    if (rc != ORC_OK) goto done;
    {
        double omega_c = o->omega_c;
        if (o->inner == ORC_CIMMINO && !(omega_c > 0.0)) {
            double lam = orc_power_lambda(m, n, rp, ci, ah, 20);
            omega_c = lam > 0.0 ? 1.0 / lam : 1.0;
        }
        int64_t kmax = o->kmax > 0 ? o->kmax : m;
        if (o->krylov == ORC_CGNE)
            rc = cgne(o, m, n, rp, ci, ah, perm, omega_c, fh, eps, kmax, dw, dyh, info);
        else if (o->krylov == ORC_MRNE)
            rc = mrne(o, m, n, rp, ci, ah, perm, omega_c, fh, eps, kmax, dw, dyh, info);
        else if (o->krylov == ORC_BAGMRES)
            rc = bagmres(o, m, n, rp, ci, ah, perm, omega_c, fh, eps, kmax, dw, dyh, info);
        else
            rc = abgmres(o, m, n, rp, ci, ah, perm, omega_c, fh, eps, kmax, dw, dyh, info);
        info->omega_c = omega_c;
    }
    if (rc != ORC_OK) goto done;
    csr_mv(m, rp, ci, ah, dw, r);
    for (int64_t i = 0; i < m; ++i) r[i] = fh[i] - r[i];
    info->res_true = nrm2(m, r);
    if (dy)
        for (int64_t i = 0; i < m; ++i) dy[i] = dyh[i] / rho[i];
done:
    free(rho); free(ah); free(fh); free(dyh); free(r); free(perm);
    return rc;
}

/* ----------------------------------------------------------------------------------- */
/* Predictor stage (eq. step_predictor): with d = sqrt(x/s) and r_d = c - A^T y - s,     */
/*   f_af = b + A (d^2 o r_d);  dw_af from the min-norm solve;                          */
/*   ds_af = r_d - dw_af / d;   dx_af = -d^2 o ds_af - x;   dy_af from the multipliers. */
int orc_affine_direction(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci,
                         const double* val, const double* b, const double* c, const double* x,
                         const double* y, const double* s, double eps, const orc_solver_opts* o,
                         double* dx, double* dy, double* ds, orc_krylov_info* info) {
    double* d = (double*)malloc((size_t)n * sizeof(double));
    double* rd = (double*)malloc((size_t)n * sizeof(double));
    double* t = (double*)malloc((size_t)n * sizeof(double));
    double* f = (double*)malloc((size_t)m * sizeof(double));
    double* dw = (double*)malloc((size_t)n * sizeof(double));
    int rc = ORC_ENOMEM;
    if (!d || !rd || !t || !f || !dw) goto done;
    for (int64_t j = 0; j < n; ++j) d[j] = sqrt(x[j] / s[j]);
    csr_tmv(m, n, rp, ci, val, y, rd);
    for (int64_t j = 0; j < n; ++j) rd[j] = c[j] - rd[j] - s[j];
    for (int64_t j = 0; j < n; ++j) t[j] = d[j] * d[j] * rd[j];
    csr_mv(m, rp, ci, val, t, f);
    for (int64_t i = 0; i < m; ++i) f[i] = b[i] + f[i];
    rc = orc_dirsolve(m, n, rp, ci, val, d, f, eps, o, dw, dy, info);
    if (rc != ORC_OK) goto done;
    for (int64_t j = 0; j < n; ++j) ds[j] = rd[j] - dw[j] / d[j];
    for (int64_t j = 0; j < n; ++j) dx[j] = -d[j] * d[j] * ds[j] - x[j];
done:
    free(d); free(rd); free(t); free(f); free(dw);
    return rc;
}

/* Corrector stage (eq. step_corrector), centring term sigma*mu:                         */
/*   f_cc = A ((dx_af o ds_af - sigma mu) / s);  dw_cc from the min-norm solve;          */
/*   ds_cc = -dw_cc / d;  dx_cc = -d^2 o ds_cc - (dx_af o ds_af)/s + sigma mu / s.       */
int orc_corrector_direction(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci,
                            const double* val, const double* x, const double* s,
                            const double* dx_af, const double* ds_af, double sigma_mu,
                            double eps, const orc_solver_opts* o, double* dx, double* dy,
                            double* ds, orc_krylov_info* info) {
    double* d = (double*)malloc((size_t)n * sizeof(double));
    double* t = (double*)malloc((size_t)n * sizeof(double));
    double* f = (double*)malloc((size_t)m * sizeof(double));
    double* dw = (double*)malloc((size_t)n * sizeof(double));
    int rc = ORC_ENOMEM;
    if (!d || !t || !f || !dw) goto done;
    for (int64_t j = 0; j < n; ++j) d[j] = sqrt(x[j] / s[j]);
    for (int64_t j = 0; j < n; ++j) t[j] = (dx_af[j] * ds_af[j] - sigma_mu) / s[j];
    csr_mv(m, rp, ci, val, t, f);
    rc = orc_dirsolve(m, n, rp, ci, val, d, f, eps, o, dw, dy, info);
    if (rc != ORC_OK) goto done;
    for (int64_t j = 0; j < n; ++j) ds[j] = -dw[j] / d[j];
    for (int64_t j = 0; j < n; ++j)
        dx[j] = -d[j] * d[j] * ds[j] - (dx_af[j] * ds_af[j]) / s[j] + sigma_mu / s[j];
done:
    free(d); free(t); free(f); free(dw);
    return rc;
}

/* A centrality corrector (multiple centrality correctors of Gondzio, the multi-corrector */
/* framework the paper names in its comparison with MOSEK): the direction with          */
/* A dx = 0, A^T dy + ds = 0 and S dx + X ds = r for a complementarity target r, solved  */
/* like the corrector of Sec. 2.2: f = A t with t = -r/s, min ||dw|| s.t. (A D) dw = f,  */
/* then ds = -dw/d and dx = -d^2 ds - t.                                                 */
int orc_centrality_direction(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci,
                             const double* val, const double* x, const double* s, const double* r,
                             double eps, const orc_solver_opts* o, double* dx, double* dy, double* ds,
                             orc_krylov_info* info) {
    double* d = (double*)malloc((size_t)n * sizeof(double));
    double* t = (double*)malloc((size_t)n * sizeof(double));
    double* f = (double*)malloc((size_t)m * sizeof(double));
    double* dw = (double*)malloc((size_t)n * sizeof(double));
    int rc = ORC_ENOMEM;
    if (!d || !t || !f || !dw) goto done;
    for (int64_t j = 0; j < n; ++j) d[j] = sqrt(x[j] / s[j]);
    for (int64_t j = 0; j < n; ++j) t[j] = -r[j] / s[j];
    csr_mv(m, rp, ci, val, t, f);
    rc = orc_dirsolve(m, n, rp, ci, val, d, f, eps, o, dw, dy, info);
    if (rc != ORC_OK) goto done;
    for (int64_t j = 0; j < n; ++j) ds[j] = -dw[j] / d[j];
    for (int64_t j = 0; j < n; ++j) dx[j] = -d[j] * d[j] * ds[j] - t[j];
done:
    free(d); free(t); free(f); free(dw);
    return rc;
}

/* Gondzio's corrector parameters: aspiration step increase, acceptance fraction of it,  */
/* and the box [BMIN, BMAX] sigma mu for the target complementarity products            */
#define MCC_DELTA 0.1
#define MCC_GAMMA 0.1
#define MCC_BMIN 0.1
#define MCC_BMAX 10.0

/* The complementarity target of a centrality corrector at the trial point of the       */
/* aspiration step lengths tp, td along (dx, ds): v = (x + tp dx)(s + td ds), each       */
/* product moved into [BMIN, BMAX] sigma mu, the decrease of large products capped at   */
/* BMAX sigma mu: r = clip(v) - v, r >= -BMAX sigma mu.                                 */
void orc_centrality_target(int64_t n, const double* x, const double* s, const double* dx,
                           const double* ds, double tp, double td, double sigma_mu, double* r) {
    const double lo = MCC_BMIN * sigma_mu, hi = MCC_BMAX * sigma_mu;
    for (int64_t j = 0; j < n; ++j) {
        const double v = (x[j] + tp * dx[j]) * (s[j] + td * ds[j]);
        double vt = v;
        if (vt < lo) vt = lo;
        if (vt > hi) vt = hi;
        double rj = vt - v;
        if (rj < -hi) rj = -hi;
        r[j] = rj;
    }
}

/* ----------------------------------------------------------------------------------- */
/* Starting point: Mehrotra's heuristic, with both least-squares solves done by the     */
/* same min-norm solver at D = I (so rank-deficient A needs no preprocessing):          */
/*   x~ = min-norm solution of A x = b;  A^T y~ = projection of c onto R(A^T);          */
/*   s~ = c - A^T y~;  shift x~, s~ into the positive orthant and balance them.          */
int orc_init_point(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                   const double* b, const double* c, const orc_solver_opts* o, double tol,
                   double* x, double* y, double* s) {
    orc_krylov_info info;
    double* f = (double*)malloc((size_t)m * sizeof(double));
    double* w = (double*)malloc((size_t)n * sizeof(double));
    int rc = ORC_ENOMEM;
    if (!f || !w) goto done;
    rc = orc_dirsolve(m, n, rp, ci, val, NULL, b, tol, o, x, NULL, &info);
    if (rc != ORC_OK) goto done;
    csr_mv(m, rp, ci, val, c, f);
    rc = orc_dirsolve(m, n, rp, ci, val, NULL, f, tol, o, w, y, &info);
    if (rc != ORC_OK) goto done;
    for (int64_t j = 0; j < n; ++j) s[j] = c[j] - w[j];
    {
        double xmin = x[0], smin = s[0];
        for (int64_t j = 1; j < n; ++j) { if (x[j] < xmin) xmin = x[j]; if (s[j] < smin) smin = s[j]; }
        double dxs = -1.5 * xmin > 0.0 ? -1.5 * xmin : 0.0;
        double dss = -1.5 * smin > 0.0 ? -1.5 * smin : 0.0;
        for (int64_t j = 0; j < n; ++j) { x[j] += dxs; s[j] += dss; }
        double xs = dot(n, x, s), sx = 0.0, ss = 0.0;
        for (int64_t j = 0; j < n; ++j) { sx += x[j]; ss += s[j]; }
        double hx = 0.5 * xs / ss, hs = 0.5 * xs / sx;
        for (int64_t j = 0; j < n; ++j) { x[j] += hx; s[j] += hs; }
        for (int64_t j = 0; j < n; ++j)
            if (!(x[j] > 0.0) || !(s[j] > 0.0)) { rc = ORC_EINVAL; goto done; }
    }
done:
    free(f); free(w);
    return rc;
}

/* ----------------------------------------------------------------------------------- */
/* step length by the ratio test (eq. steplength): min(1, eta * min_{dv_i<0} -v_i/dv_i) */
static double ratio(int64_t n, const double* v, const double* dv, double eta) {
    double a = INFINITY;
    for (int64_t j = 0; j < n; ++j)
        if (dv[j] < 0.0) { double t = -v[j] / dv[j]; if (t < a) a = t; }
    a = eta * a;
    return a < 1.0 ? a : 1.0;
}

/* the IPM state carried between iterations */
typedef struct {
    double eps_in;
    int32_t fail_prev;
    int32_t k;
} orc_ipm_state;

/* the paper's error measure (eq. errorMeasureDef) and the relative version used for the */
/* stopping test (relative duality gap in place of mu)                                   */
static void measures(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                     const double* b, const double* c, const double* x, const double* y,
                     const double* s, double* rpv, double* rdv, orc_iter_log* L) {
    csr_mv(m, rp, ci, val, x, rpv);
    for (int64_t i = 0; i < m; ++i) rpv[i] = b[i] - rpv[i];
    csr_tmv(m, n, rp, ci, val, y, rdv);
    for (int64_t j = 0; j < n; ++j) rdv[j] = c[j] - rdv[j] - s[j];
    double nb = nrm2(m, b), nc = nrm2(n, c);
    double mu = dot(n, x, s) / (double)n;
    double rp_rel = nrm2(m, rpv) / (nb > 1.0 ? nb : 1.0);
    double rd_rel = nrm2(n, rdv) / (nc > 1.0 ? nc : 1.0);
    double pobj = dot(n, c, x), dobj = dot(m, b, y);
    double gap_rel = fabs(pobj - dobj) / (fabs(pobj) > 1.0 ? fabs(pobj) : 1.0);
    double g = mu; if (rp_rel > g) g = rp_rel; if (rd_rel > g) g = rd_rel;
    double gr = gap_rel; if (rp_rel > gr) gr = rp_rel; if (rd_rel > gr) gr = rd_rel;
    L->mu = mu; L->gamma = g; L->gamma_rel = gr; L->rp_rel = rp_rel; L->rd_rel = rd_rel;
    L->gap_rel = gap_rel; L->pobj = pobj; L->dobj = dobj;
}

/* One iteration of Mehrotra's predictor-corrector algorithm from (x, y, s).            */
/* Returns 1 in *done if the stopping test held at the entry point (no step taken).     */
int orc_ipm_iterate(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                    const double* b, const double* c, const orc_ipm_opts* op, double* x,
                    double* y, double* s, orc_ipm_state* st, orc_iter_log* L, int32_t* done) {
    double *rpv = 0, *rdv = 0, *dxa = 0, *dya = 0, *dsa = 0, *dxc = 0, *dyc = 0, *dsc = 0;
    int rc = ORC_ENOMEM;
    memset(L, 0, sizeof(*L));
    *done = 0;
    rpv = (double*)malloc((size_t)m * sizeof(double));
    rdv = (double*)malloc((size_t)n * sizeof(double));
    dxa = (double*)malloc((size_t)n * sizeof(double));
    dya = (double*)malloc((size_t)m * sizeof(double));
    dsa = (double*)malloc((size_t)n * sizeof(double));
    dxc = (double*)malloc((size_t)n * sizeof(double));
    dyc = (double*)malloc((size_t)m * sizeof(double));
    dsc = (double*)malloc((size_t)n * sizeof(double));
    if (!rpv || !rdv || !dxa || !dya || !dsa || !dxc || !dyc || !dsc) goto done;
    measures(m, n, rp, ci, val, b, c, x, y, s, rpv, rdv, L);
    if (L->gamma_rel <= op->eps_out) { *done = 1; rc = ORC_OK; goto done; }
    /* eps_in schedule (Sec. 4.2): tightened by 0.75 while log10(Gamma) is in (-3, 1],   */
    /* by 0.375 once it is <= -3, unchanged above 1; times 1.5 after a failed solve;      */
    /* kept in [eps_in_min, eps_in_max]                                                  */
    if (st->k >= 1) {
        double lg = log10(L->gamma);
        double fac = 1.0;
        if (lg <= -3.0) fac = 0.375;
        else if (lg <= 1.0) fac = 0.75;
        if (st->fail_prev) fac *= 1.5;
        st->eps_in *= fac;
    }
    if (st->eps_in < op->eps_in_min) st->eps_in = op->eps_in_min;
    if (st->eps_in > op->eps_in_max) st->eps_in = op->eps_in_max;
    L->eps_in = st->eps_in;
    {
        orc_krylov_info ia, ic;
        memset(&ic, 0, sizeof(ic));
        rc = orc_affine_direction(m, n, rp, ci, val, b, c, x, y, s, st->eps_in, &op->solver,
                                  dxa, dya, dsa, &ia);
        if (rc != ORC_OK) goto done;
        L->k_af = ia.iters; L->res_af = ia.beta > 0 ? ia.res_true / ia.beta : 0.0; L->fail_af = ia.failed;
        double ap = ratio(n, x, dxa, op->eta), ad = ratio(n, s, dsa, op->eta);
        double sigma = 0.0;
        if (ap < 1.0 || ad < 1.0) {
            double mu_af = 0.0;
            for (int64_t j = 0; j < n; ++j) mu_af += (x[j] + ap * dxa[j]) * (s[j] + ad * dsa[j]);
            mu_af /= (double)n;
            if (L->gamma > 1e-3) {
                double r = mu_af / L->mu;
                sigma = r * r;
            } else {
                sigma = 10.0 * L->gamma;
            }
            if (sigma > op->sigma_max) sigma = op->sigma_max;
            rc = orc_corrector_direction(m, n, rp, ci, val, x, s, dxa, dsa, sigma * L->mu,
                                         st->eps_in, &op->solver, dxc, dyc, dsc, &ic);
            if (rc != ORC_OK) goto done;
            for (int64_t j = 0; j < n; ++j) { dxa[j] += dxc[j]; dsa[j] += dsc[j]; }
            for (int64_t i = 0; i < m; ++i) dya[i] += dyc[i];
            L->k_cc = ic.iters; L->res_cc = ic.beta > 0 ? ic.res_true / ic.beta : 0.0; L->fail_cc = ic.failed;
        }
        L->sigma = sigma;
        /* trial step lengths, then joint geometric back-tracking until the centrality  */
        /* condition min_i x_i s_i >= phi x^T s / n holds at the new point              */
        ap = ratio(n, x, dxa, op->eta);
        ad = ratio(n, s, dsa, op->eta);
        /* multiple centrality correctors: while a step length is short of 1, aim at     */
        /* step lengths larger by MCC_DELTA, move the products at that trial point into  */
        /* the box around sigma mu, and keep the corrected direction when its shorter    */
        /* step length grows by at least MCC_GAMMA MCC_DELTA; stop at the first miss     */
        if (op->max_correctors > 0 && sigma > 0.0) {
            double* r = (double*)malloc((size_t)n * sizeof(double));
            double* dxk = (double*)malloc((size_t)n * sizeof(double));
            double* dsk = (double*)malloc((size_t)n * sizeof(double));
            double* dyk = (double*)malloc((size_t)m * sizeof(double));
            double* tx = (double*)malloc((size_t)n * sizeof(double));
            double* ts = (double*)malloc((size_t)n * sizeof(double));
            rc = ORC_ENOMEM;
            if (r && dxk && dsk && dyk && tx && ts) {
                rc = ORC_OK;
                for (int32_t q = 0; q < op->max_correctors; ++q) {
                    if (ap >= 1.0 && ad >= 1.0) break;
                    const double tp = fmin(1.0, ap + MCC_DELTA), td = fmin(1.0, ad + MCC_DELTA);
                    orc_centrality_target(n, x, s, dxa, dsa, tp, td, sigma * L->mu, r);
                    orc_krylov_info ik;
                    rc = orc_centrality_direction(m, n, rp, ci, val, x, s, r, st->eps_in, &op->solver,
                                                  dxk, dyk, dsk, &ik);
                    if (rc != ORC_OK) break;
                    for (int64_t j = 0; j < n; ++j) { tx[j] = dxa[j] + dxk[j]; ts[j] = dsa[j] + dsk[j]; }
                    const double ap2 = ratio(n, x, tx, op->eta), ad2 = ratio(n, s, ts, op->eta);
                    if (fmin(ap2, ad2) < fmin(ap, ad) + MCC_GAMMA * MCC_DELTA) break;
                    memcpy(dxa, tx, (size_t)n * sizeof(double));
                    memcpy(dsa, ts, (size_t)n * sizeof(double));
                    for (int64_t i = 0; i < m; ++i) dya[i] += dyk[i];
                    ap = ap2;
                    ad = ad2;
                    L->correctors += 1;
                }
            }
            free(r); free(dxk); free(dsk); free(dyk); free(tx); free(ts);
            if (rc != ORC_OK) goto done;
        }
        int32_t t = 0;
        for (;;) {
            double mn = INFINITY, sum = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double pr = (x[j] + ap * dxa[j]) * (s[j] + ad * dsa[j]);
                if (pr < mn) mn = pr;
                sum += pr;
            }
            if (mn >= op->phi * sum / (double)n || t >= op->max_backtrack) break;
            ap *= op->backtrack;
            ad *= op->backtrack;
            ++t;
        }
        L->alpha_p = ap; L->alpha_d = ad; L->backtracks = t;
        for (int64_t j = 0; j < n; ++j) { x[j] += ap * dxa[j]; s[j] += ad * dsa[j]; }
        for (int64_t i = 0; i < m; ++i) y[i] += ad * dya[i];
        st->fail_prev = ia.failed || ic.failed;
        st->k += 1;
        for (int64_t j = 0; j < n; ++j)
            if (!isfinite(x[j]) || !isfinite(s[j]) || !(x[j] > 0.0) || !(s[j] > 0.0)) { rc = ORC_DIVERGED; goto done; }
    }
    rc = ORC_OK;
done:
    free(rpv); free(rdv); free(dxa); free(dya); free(dsa); free(dxc); free(dyc); free(dsc);
    return rc;
}

void orc_ipm_opts_default(orc_ipm_opts* op) {
    memset(op, 0, sizeof(*op));
    op->solver.krylov = ORC_ABGMRES;
    op->solver.inner = ORC_NESOR;
    op->solver.ell = 2;
    op->solver.order = ORC_ORDER_COLOUR;
    op->solver.flexible = 0;
    op->solver.omega = 1.0;
    op->solver.omega_c = 0.0;
    op->solver.kmax = 0;
    op->max_iter = 99;
    op->start = 0;
    op->eps_out = 1e-8;
    op->eta = 0.9995;
    op->phi = 1e-5;
    op->sigma_max = 0.208;
    op->eps_in0 = 1e-6;
    op->eps_in_min = 1e-14;
    op->eps_in_max = 1e-4;
    op->init_tol = 1e-10;
    op->backtrack = 0.95;
    op->max_backtrack = 200;
}

/* Split free variables x_j = x+_j - x-_j (the bounded-variable reduction to standard   */
/* form): both parts grow without bound along the central path, since the two dual     */
/* slacks of a pair must both vanish.  After the starting point and after every step,   */
/* a pair whose smaller part exceeds (1 + |x+ - x-|) / 2 is lowered by the excess, both  */
/* parts by the same amount, which leaves x_j, A x and c^T x unchanged.  pairs holds    */
/* the two column indices of each pair.                                                */
static void recentre_pairs(int64_t npairs, const int64_t* pairs, double* x) {
    for (int64_t t = 0; t < npairs; ++t) {
        const int64_t p = pairs[2 * t], q = pairs[2 * t + 1];
        const double a = x[p], b = x[q];
        const double lo = a < b ? a : b;
        const double cap = 0.5 * (1.0 + fabs(a - b));
        if (lo > cap) {
            const double d = lo - cap;
            x[p] = a - d;
            x[q] = b - d;
        }
    }
}

/* The interior-point loop.  x, y, s are outputs (and inputs when op->start == 1).      */
/* log may hold max_iter + 1 entries or be NULL.  Returns ORC_OK (stopping test met),   */
/* ORC_NOT_CONVERGED (iteration limit) or ORC_DIVERGED (non-finite or non-positive).    */
/* npairs > 0: the split free variables to recentre (recentre_pairs).                  */
int orc_ipm_pairs(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                  const double* b, const double* c, const orc_ipm_opts* op, int64_t npairs,
                  const int64_t* pairs, double* x, double* y, double* s, orc_iter_log* log,
                  int32_t* iters, double* gamma_out, double* gamma_rel_out) {
    int rc;
    if (op->start == 0) {
        rc = orc_init_point(m, n, rp, ci, val, b, c, &op->solver, op->init_tol, x, y, s);
        if (rc != ORC_OK) return rc;
        recentre_pairs(npairs, pairs, x);
    }
    orc_ipm_state st;
    st.eps_in = op->eps_in0;
    st.fail_prev = 0;
    st.k = 0;
    orc_iter_log L;
    for (int32_t k = 0; k <= op->max_iter; ++k) {
        int32_t done = 0;
        if (k == op->max_iter) {
            /* evaluate the final point only */
            double* rpv = (double*)malloc((size_t)m * sizeof(double));
            double* rdv = (double*)malloc((size_t)n * sizeof(double));
            memset(&L, 0, sizeof(L));
            measures(m, n, rp, ci, val, b, c, x, y, s, rpv, rdv, &L);
            free(rpv); free(rdv);
            if (log) log[k] = L;
            *iters = k;
            *gamma_out = L.gamma;
            *gamma_rel_out = L.gamma_rel;
            return L.gamma_rel <= op->eps_out ? ORC_OK : ORC_NOT_CONVERGED;
        }
        rc = orc_ipm_iterate(m, n, rp, ci, val, b, c, op, x, y, s, &st, &L, &done);
        if (log) log[k] = L;
        *iters = k;
        *gamma_out = L.gamma;
        *gamma_rel_out = L.gamma_rel;
        if (rc != ORC_OK) return rc;
        if (done) return ORC_OK;
        recentre_pairs(npairs, pairs, x);
    }
    return ORC_NOT_CONVERGED;
}

int orc_ipm(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
            const double* b, const double* c, const orc_ipm_opts* op, double* x, double* y,
            double* s, orc_iter_log* log, int32_t* iters, double* gamma_out, double* gamma_rel_out) {
    return orc_ipm_pairs(m, n, rp, ci, val, b, c, op, 0, NULL, x, y, s, log, iters, gamma_out, gamma_rel_out);
}
