// Mehrotra's predictor-corrector interior-point iteration (Sec. 2.1) driven from the
// host with every vector operation on the device.  The host holds only the scalars the
// algorithm branches on (mu, the error measure, step lengths, sigma); each comes back
// through one small pinned read after a fixed-order device reduction.
#include <math.h>

#include <algorithm>

#include "lpk_impl.h"

namespace lpk {

// starting point (the paper uses LIPSOL's; this is Mehrotra's published heuristic): both
// least-squares problems are min-norm solves at D = I with the same Krylov solver, so
// rank-deficient A needs no preprocessing.
//   x~ = argmin ||x|| s.t. A x = b;  A^T y~ = projection of c on R(A^T);  s~ = c - A^T y~
//   shift x~, s~ to positive, then balance them by 1/2 x^T s / sum(s), 1/2 x^T s / sum(x)
lp_status ipm_init_point(lp_problem* p) {
    hipStream_t st = p->st;
    const int64_t m = p->m, n = p->n;
    lp_status rc = build_scaling(p, nullptr);
    if (rc != LP_OK) return rc;
    lp_krylov_info ki;
    const double tol = p->opt.init_tol;
    // x~ from b
    rc = krylov_solve(p, p->b, tol, p->x, p->dyh, &ki);
    if (rc != LP_OK) return rc;
    // f = A c, then w = projection of c, y~ = dyh / rho
    spmv_f64(st, p->g_csr, (int)m, p->rp, p->ci, p->a, p->c, p->f, EPI_PLAIN, nullptr, nullptr, nullptr);
    rc = krylov_solve(p, p->f, tol, p->dw, p->dyh, &ki);
    if (rc != LP_OK) return rc;
    div_by(st, m, p->dyh, p->rho, p->y);
    lincomb(st, n, 1.0, p->c, -1.0, p->dw, p->s);
    min2(st, p->red, n, p->x, p->s);
    double mins[2];
    rc = sync_read(p, p->red.out, mins, 2);
    if (rc != LP_OK) return rc;
    const double dxs = -1.5 * mins[0] > 0.0 ? -1.5 * mins[0] : 0.0;
    const double dss = -1.5 * mins[1] > 0.0 ? -1.5 * mins[1] : 0.0;
    shift2(st, p->red, n, p->x, p->s, dxs, dss);
    double q[3];
    rc = sync_read(p, p->red.out, q, 3);
    if (rc != LP_OK) return rc;
    const double hx = 0.5 * q[0] / q[2], hs = 0.5 * q[0] / q[1];
    shift2(st, p->red, n, p->x, p->s, hx, hs);
    min2(st, p->red, n, p->x, p->s);
    rc = sync_read(p, p->red.out, mins, 2);
    if (rc != LP_OK) return rc;
    if (!(mins[0] > 0.0) || !(mins[1] > 0.0)) {
        set_error("starting point is not strictly positive");
        return LP_DIVERGED;
    }
    p->have_point = true;
    p->ist.eps_in = p->opt.eps_in0;
    p->ist.k = 0;
    p->ist.fail_prev = 0;
    return LP_OK;
}

// residuals r_p = b - A x, r_d = c - A^T y - s and the scalars of the error measure
// (eq. errorMeasureDef) and of the relative stopping test
static lp_status measures(lp_problem* p, lp_iter_info* L) {
    hipStream_t st = p->st;
    const int64_t m = p->m, n = p->n;
    spmv_f64(st, p->g_csr, (int)m, p->rp, p->ci, p->a, p->x, p->rpv, EPI_B_MINUS, p->b, nullptr, nullptr);
    spmv_f64(st, p->g_csc, (int)n, p->cp, p->ri, p->ac, p->y, p->rdv, EPI_B1_MINUS_B2, p->c, p->s, nullptr);
    ipm_measures(st, p->red, m, n, p->x, p->s, p->c, p->rdv, p->b, p->y, p->rpv);
    double q[5];
    lp_status rc = sync_read(p, p->red.out, q, 5);
    if (rc != LP_OK) return rc;
    const double nb = p->norm_b, nc = p->norm_c;
    L->mu = q[0] / (double)n;
    L->rp_rel = std::sqrt(q[4]) / (nb > 1.0 ? nb : 1.0);
    L->rd_rel = std::sqrt(q[2]) / (nc > 1.0 ? nc : 1.0);
    L->pobj = q[1];
    L->dobj = q[3];
    L->gap_rel = std::fabs(q[1] - q[3]) / (std::fabs(q[1]) > 1.0 ? std::fabs(q[1]) : 1.0);
    L->gamma = std::max(L->mu, std::max(L->rp_rel, L->rd_rel));
    L->gamma_rel = std::max(L->gap_rel, std::max(L->rp_rel, L->rd_rel));
    return LP_OK;
}

lp_status ipm_evaluate(lp_problem* p, lp_iter_info* L) {
    *L = lp_iter_info{};
    lp_status rc = measures(p, L);
    if (rc != LP_OK) return rc;
    L->converged = L->gamma_rel <= p->opt.eps_out ? 1 : 0;
    return LP_OK;
}

static double step_from(double minratio, double eta) {
    const double a = eta * minratio;
    return a < 1.0 ? a : 1.0;
}

lp_status ipm_iterate(lp_problem* p, lp_iter_info* L) {
    hipStream_t st = p->st;
    const int64_t m = p->m, n = p->n;
    const lp_options& o = p->opt;
    *L = lp_iter_info{};
    lp_status rc = measures(p, L);
    if (rc != LP_OK) return rc;
    if (!std::isfinite(L->gamma_rel)) {
        set_error("non-finite residuals");
        return LP_DIVERGED;
    }
    if (L->gamma_rel <= o.eps_out) {
        L->converged = 1;
        return LP_OK;
    }
    // eps_in schedule of Sec. 4.2 (x0.75 while log10 Gamma in (-3, 1], x0.375 at or below
    // -3, x1.5 after a failed solve), clamped to [eps_in_min, eps_in_max]
    if (p->ist.k >= 1) {
        const double lg = std::log10(L->gamma);
        double fac = 1.0;
        if (lg <= -3.0) fac = 0.375;
        else if (lg <= 1.0) fac = 0.75;
        if (p->ist.fail_prev) fac *= 1.5;
        p->ist.eps_in *= fac;
    }
    p->ist.eps_in = std::min(std::max(p->ist.eps_in, o.eps_in_min), o.eps_in_max);
    L->eps_in = p->ist.eps_in;

    // D = diag(sqrt(x/s)); A_hat for the predictor and the corrector (same matrix)
    ipm_scaling(st, n, p->x, p->s, p->rdv, p->d, p->tn);
    rc = build_scaling(p, p->d);
    if (rc != LP_OK) return rc;
    // predictor: f_af = b + A (d^2 o r_d)
    spmv_f64(st, p->g_csr, (int)m, p->rp, p->ci, p->a, p->tn, p->f, EPI_B_PLUS, p->b, nullptr, nullptr);
    lp_krylov_info ka{}, kc{};
    rc = krylov_solve(p, p->f, p->ist.eps_in, p->dw, p->dyh, &ka);
    if (rc != LP_OK) return rc;
    L->k_af = ka.iters;
    L->res_af = ka.beta > 0.0 ? ka.res_true / ka.beta : 0.0;
    L->fail_af = ka.failed;
    div_by(st, m, p->dyh, p->rho, p->dya);
    ipm_recover_af(st, p->red, n, p->rdv, p->dw, p->d, p->x, p->s, p->dsa, p->dxa);
    double r2[2];
    rc = sync_read(p, p->red.out, r2, 2);
    if (rc != LP_OK) return rc;
    double ap = step_from(r2[0], o.eta), ad = step_from(r2[1], o.eta);
    double sigma = 0.0;
    if (ap < 1.0 || ad < 1.0) {
        ipm_mu_af(st, p->red, n, p->x, p->s, p->dxa, p->dsa, ap, ad);
        double sx;
        rc = sync_read(p, p->red.out, &sx, 1);
        if (rc != LP_OK) return rc;
        const double mu_af = sx / (double)n;
        if (L->gamma > 1e-3) {
            const double r = mu_af / L->mu;
            sigma = r * r;
        } else {
            sigma = 10.0 * L->gamma;
        }
        if (sigma > o.sigma_max) sigma = o.sigma_max;
        const double smu = sigma * L->mu;
        // corrector: f_cc = A ((dx_af o ds_af - sigma mu) / s)
        ipm_cc_rhs(st, n, p->dxa, p->dsa, p->s, smu, p->tn);
        spmv_f64(st, p->g_csr, (int)m, p->rp, p->ci, p->a, p->tn, p->f, EPI_PLAIN, nullptr, nullptr, nullptr);
        rc = krylov_solve(p, p->f, p->ist.eps_in, p->dw, p->dyh, &kc);
        if (rc != LP_OK) return rc;
        L->k_cc = kc.iters;
        L->res_cc = kc.beta > 0.0 ? kc.res_true / kc.beta : 0.0;
        L->fail_cc = kc.failed;
        div_by(st, m, p->dyh, p->rho, p->dyc);
        axpy(st, m, 1.0, p->dyc, p->dya);
        ipm_recover_cc(st, p->red, n, p->dw, p->d, p->x, p->s, smu, p->dxa, p->dsa);
        rc = sync_read(p, p->red.out, r2, 2);
        if (rc != LP_OK) return rc;
        ap = step_from(r2[0], o.eta);
        ad = step_from(r2[1], o.eta);
    }
    L->sigma = sigma;
    // back-tracking until min_i x_i s_i >= phi x^T s / n at the new point (Sec. 2.1)
    int32_t t = 0;
    for (;;) {
        ipm_backtrack(st, p->red, n, p->x, p->s, p->dxa, p->dsa, ap, ad);
        rc = sync_read(p, p->red.out, r2, 2);
        if (rc != LP_OK) return rc;
        if (r2[0] >= o.phi * r2[1] / (double)n || t >= o.max_backtrack) break;
        ap *= o.backtrack;
        ad *= o.backtrack;
        ++t;
    }
    L->alpha_p = ap;
    L->alpha_d = ad;
    L->backtracks = t;
    ipm_update(st, p->red, m, n, p->x, p->s, p->y, p->dxa, p->dsa, p->dya, ap, ad);
    double bad;
    rc = sync_read(p, p->red.out, &bad, 1);
    if (rc != LP_OK) return rc;
    p->ist.fail_prev = (ka.failed || kc.failed) ? 1 : 0;
    p->ist.k += 1;
    if (bad > 0.0) {
        set_error("iterate left the positive orthant or became non-finite");
        return LP_DIVERGED;
    }
    return LP_OK;
}

}  // namespace lpk
