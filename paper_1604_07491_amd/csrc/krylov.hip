// The search-direction solve on the device: AB-GMRES right-preconditioned by inner
// iterations (Sec. 3.2) on the row-scaled min-norm problem (Sec. 3.5).
//
// Differences from the paper's CPU layout, all exact in exact arithmetic:
//  * flexible final step: the multiplier vectors p_k of every preconditioner application
//    are kept (P = [p_1 .. p_k]) and the solution is dw = A_hat^T (P y); z_k = A_hat^T p_k
//    is recomputed in FP64, so the Arnoldi relation and dw in R(A_hat^T) hold to FP64 even
//    when the sweeps run in FP32.  The multipliers also give dy = diag(rho)^-1 P y with no
//    extra matrix-vector product.
//  * classical Gram-Schmidt applied twice in place of modified Gram-Schmidt (Sec. 3.2 uses
//    MGS); both orthogonalise to working precision, CGS2 in two reductions per pass.
//  * the Hessenberg least-squares problem is kept in QR form by Givens rotations on the
//    device; the host only polls the convergence flag every few iterations.
#include <algorithm>

#include "lpk_impl.h"

namespace lpk {

lp_status sync_read(lp_problem* p, const double* dev, double* host, int count) {
    LPK_HIP(hipMemcpyAsync(p->host_out, dev, sizeof(double) * count, hipMemcpyDeviceToHost, p->st));
    LPK_HIP(hipStreamSynchronize(p->st));
    for (int i = 0; i < count; ++i) host[i] = p->host_out[i];
    return LP_OK;
}

static lp_status read_ctl(lp_problem* p, KrylovCtl* out) {
    LPK_HIP(hipMemcpyAsync(p->host_ctl, p->ctl, sizeof(KrylovCtl), hipMemcpyDeviceToHost, p->st));
    LPK_HIP(hipStreamSynchronize(p->st));
    *out = *p->host_ctl;
    return LP_OK;
}

// Dense path, once per scaling: G = A_hat A_hat^T (MFMA), then the inner-iteration
// preconditioner in the matrix form of Sec. 3.1/3.2, C<l> = sum_{i<l} H^i M^-1 with the SOR
// splitting M = I/omega + tril(G, -1) (unit diagonal, Sec. 3.5) and H = I - M^-1 G:
//   X = M^-1 by block forward substitution (64-row blocks: R = I - G[B, <B] X[<B, :] by
//   GEMM, then the diagonal block's substitution), C_1 = X, C_{i+1} = X + C_i - X (G C_i).
// l SOR sweeps from zero apply exactly this C to v, so each Krylov iteration needs only
// p = C v and u = G p.
static lp_status build_dense_preconditioner(lp_problem* p) {
    hipStream_t st = p->st;
    const int m = (int)p->m;
    const int64_t mm = (int64_t)m * m;
    const bool mixed = p->opt.precision == LP_MIXED;
    const double om = p->opt.omega;
    const int ell = std::max(1, (int)p->opt.inner_sweeps);
    const double nbt = (double)((m + 63) / 64);
    double fl = 2.0 * (double)p->n * 64.0 * 64.0 * nbt * (nbt + 1.0) / 2.0;     // Gram tiles
    fl += (double)m * m * m / 3.0 * 2.0 + (ell - 1) * 4.0 * (double)m * m * m;   // M^-1 and C
    Prof pr(p, LP_K_GRAM, -1, 8.0 * (double)m * p->n + 8.0 * mm * (3.0 + 3.0 * (ell - 1)), fl);
    gram_f64(st, m, p->n, p->ah, p->n, p->G, nullptr);
    fill(st, mm, 0.0, p->Xinv);
    for (int r0 = 0; r0 < m; r0 += 64) {
        const int b = std::min(64, m - r0), ncols = r0 + b;
        // R = I[B, :] - G[B, 0:r0] X[0:r0, 0:ncols]   (K = 0 for the first block: R = I)
        gemm_f64(st, b, ncols, r0, -1.0, p->G + (int64_t)r0 * m, m, p->Xinv, m, 0.0, nullptr, nullptr, m,
                 p->Rblk, m, r0);
        trsm_diag(st, m, r0, b, p->G, p->Rblk, m, p->Xinv, om, ncols);
    }
    const double* Ccur = p->Xinv;
    double* bufs[2] = {p->Cmat, p->Tmat2};
    for (int i = 1; i < ell; ++i) {
        double* Cn = bufs[(i - 1) & 1];
        gemm_f64(st, m, m, m, 1.0, p->G, m, Ccur, m, 0.0, nullptr, nullptr, m, p->Tmat, m, -1);
        gemm_f64(st, m, m, m, -1.0, p->Xinv, m, p->Tmat, m, 1.0, p->Xinv, Ccur, m, Cn, m, -1);
        Ccur = Cn;
    }
    p->Capply = Ccur;
    if (mixed) to_f32(st, mm, Ccur, p->C32);
    LPK_HIP(hipGetLastError());
    return LP_OK;
}

// rho, A_hat (CSR, CSC; FP32 copies in mixed mode) for D = diag(d) (d NULL: D = I), and
// the Cimmino step 1/lambda when it is not fixed by the options
lp_status build_scaling(lp_problem* p, const double* d_dev) {
    hipStream_t st = p->st;
    const bool mixed = p->opt.precision == LP_MIXED;
    const bool cim = p->opt.inner == LP_CIMMINO;
    scale_rows(st, p->g_csr, (int)p->m, p->rp, p->ci, p->a, d_dev, p->rho, p->ah, mixed ? p->ah32 : nullptr);
    scale_cols(st, (int)p->n, p->cp, p->ri, p->ac, d_dev, p->rho, p->ahc, (mixed && cim) ? p->ahc32 : nullptr);
    // dense path: the CSR values of a dense A are A_hat row-major; G = A_hat A_hat^T
    if (p->gsor) {
        lp_status rc = build_dense_preconditioner(p);
        if (rc != LP_OK) return rc;
    }
    LPK_HIP(hipGetLastError());
    if (cim) {
        if (p->opt.omega_c > 0.0) {
            p->omega_c = p->opt.omega_c;
        } else {
            // 20 power iterations on A_hat A_hat^T from e / sqrt(m): lambda = ||A_hat A_hat^T v||
            double* v = p->dtmp_m;
            fill(st, p->m, 1.0 / std::sqrt((double)p->m), v);
            for (int it = 0; it < 20; ++it) {
                spmv_f64(st, p->g_csc, (int)p->n, p->cp, p->ri, p->ahc, v, p->dtmp_n, EPI_PLAIN, nullptr, nullptr, nullptr);
                spmv_f64(st, p->g_csr, (int)p->m, p->rp, p->ci, p->ah, p->dtmp_n, v, EPI_PLAIN, nullptr, nullptr, nullptr);
                sumsq(st, p->red, p->m, v);
                if (it + 1 < 20) vec_scale_by_norm(st, p->red, p->m, v, 0);
            }
            double l2;
            lp_status rc = sync_read(p, p->red.out, &l2, 1);
            if (rc != LP_OK) return rc;
            const double lam = std::sqrt(l2);
            p->omega_c = lam > 0.0 ? 1.0 / lam : 1.0;
        }
    }
    p->scaled_for_d = false;
    return LP_OK;
}

// enqueue one application of the inner-iteration preconditioner to column k of V (k and
// the done flag from ctl), with the start-of-iteration preparation when with_prep.  Each
// launch carries its algorithmic bytes for the profiler: every input and output it must
// move, each once.
void enqueue_precond(lp_problem* p, KrylovCtl* ctl, int64_t it, bool with_prep) {
    hipStream_t st = p->st;
    const bool mixed = p->opt.precision == LP_MIXED;
    const int64_t m = p->m, n = p->n, ldv = p->ldv, nnz = p->nnz;
    const int ell = std::max(1, (int)p->opt.inner_sweeps);
    const double sv = mixed ? 4.0 : 8.0;   // bytes of one A_hat value / z entry in the sweeps
    if (p->gsor) {
        if (with_prep) krylov_prep(st, m, n, p->V, p->u, p->P, ldv, nullptr, nullptr, ctl);
        {
            // l SOR sweeps on G p = v_k, applied as p = C<l> v_k
            Prof pr(p, LP_K_SWEEP, it, (double)m * m * sv + 16.0 * m);
            if (mixed)
                apply_c_f32(st, (int)m, p->C32, p->V, p->P, ldv, ctl);
            else
                apply_c_f64(st, (int)m, p->Capply, p->V, p->P, ldv, ctl);
        }
    } else if (p->opt.inner == LP_CIMMINO) {
        if (with_prep) krylov_prep(st, m, n, p->V, p->u, p->P, ldv, nullptr, nullptr, ctl);
        for (int sw = 0; sw < ell; ++sw) {
            const int first = sw == 0;
            {
                const double by = first ? m * (8.0 + sv + 16.0)
                                        : nnz * (sv + 4.0) + n * sv + m * (4.0 + 8.0 + sv + 16.0);
                Prof pr(p, LP_K_SWEEP, it, by);
                if (mixed)
                    cimmino_residual_f32(st, p->g_csr, (int)m, p->rp, p->ci, p->ah32, p->z32, p->V, p->P, ldv, p->omega_c, p->r32, first, ctl);
                else
                    cimmino_residual_f64(st, p->g_csr, (int)m, p->rp, p->ci, p->ah, p->z64, p->V, p->P, ldv, p->omega_c, p->r64, first, ctl);
            }
            if (sw + 1 < ell) {
                const double by = nnz * (sv + 4.0) + m * sv + n * (4.0 + sv * (first ? 1.0 : 2.0));
                Prof pr(p, LP_K_SWEEP, it, by);
                if (mixed)
                    cimmino_zupdate_f32(st, p->g_csc, (int)n, p->cp, p->ri, p->ahc32, p->r32, p->z32, p->omega_c, first, ctl);
                else
                    cimmino_zupdate_f64(st, p->g_csc, (int)n, p->cp, p->ri, p->ahc, p->r64, p->z64, p->omega_c, first, ctl);
            }
        }
    } else {
        if (with_prep) krylov_prep(st, m, n, p->V, p->u, p->P, ldv, mixed ? nullptr : p->z64, mixed ? p->z32 : nullptr, ctl);
        const int nc = (int)p->colours.size();
        for (int sw = 0; sw < ell; ++sw) {
            for (int c = 0; c < nc; ++c) {
                const Colour& cl = p->colours[c];
                const int wz = !(sw + 1 == ell && c + 1 == nc);
                const double by = cl.nnz * (sv + 4.0) + cl.nnz * sv * (wz ? 2.0 : 1.0) +
                                  (double)(cl.r1 - cl.r0) * (4.0 + 8.0 + 16.0);
                Prof pr(p, LP_K_SWEEP, it, by);
                if (mixed)
                    nesor_colour_f32(st, cl.g, cl.r0, cl.r1, p->rp, p->ci, p->ah32, p->z32, p->V, p->P, ldv, p->opt.omega, ctl, wz);
                else
                    nesor_colour_f64(st, cl.g, cl.r0, cl.r1, p->rp, p->ci, p->ah, p->z64, p->V, p->P, ldv, p->opt.omega, ctl, wz);
            }
        }
    }
}

// enqueue Krylov iteration `it` of the current solve (every kernel returns at once once
// ctl->done is set)
static void enqueue_iteration(lp_problem* p, int64_t it) {
    hipStream_t st = p->st;
    const int64_t m = p->m, n = p->n, ldv = p->ldv, nnz = p->nnz;
    const int32_t* skip = &p->ctl->done;
    enqueue_precond(p, p->ctl, it, true);
    if (p->gsor) {
        // u = A_hat A_hat^T p_k = G p_k
        Prof pr(p, LP_K_SPMV_CSR, it, 8.0 * m * m + 16.0 * m);
        gemv_col(st, (int)m, p->G, p->P, ldv, p->u, p->ctl);
    }
    // outer operator in FP64: z_k = A_hat^T p_k, u = A_hat z_k (dense path: u = G p_k above)
    if (!p->gsor) {
        Prof pr(p, LP_K_SPMV_CSC, it, nnz * 12.0 + m * 8.0 + n * 8.0 + (n + 1) * 4.0);
        spmv_f64_col(st, p->g_csc, (int)n, p->cp, p->ri, p->ahc, p->P, ldv, p->z64, p->ctl);
    }
    if (!p->gsor) {
        Prof pr(p, LP_K_SPMV_CSR, it, nnz * 12.0 + n * 8.0 + m * 8.0 + (m + 1) * 4.0);
        spmv_f64(st, p->g_csr, (int)m, p->rp, p->ci, p->ah, p->z64, p->u, EPI_PLAIN, nullptr, nullptr, skip);
    }
    // CGS2 + Givens; the host iteration index equals the device one while the solve runs
    const int64_t ldp = p->kmax + 1;
    const double kk = (double)(it + 1), nch = (double)p->gs.nchunks;
    {
        Prof pr(p, LP_K_GS_DOTS, it, kk * m * 8.0 + m * 8.0 + nch * kk * 8.0);
        gs_dots(st, p->gs, m, p->V, ldv, p->u, p->gpart, ldp, p->ctl);
    }
    if (p->gs_fused) {
        // each update block reduces the previous pass's partials itself (few chunks)
        {
            Prof pr(p, LP_K_GS_UPDATE, it, kk * m * 8.0 + 16.0 * m + 2.0 * nch * kk * 8.0);
            gs_update_fused(st, p->gs, m, p->V, ldv, p->u, p->gpart, p->gpart2, ldp, 0, p->H, p->ldh, p->ctl);
        }
        {
            Prof pr(p, LP_K_GS_UPDATE, it, kk * m * 8.0 + 16.0 * m + nch * kk * 8.0 + nch * 8.0);
            gs_update_fused(st, p->gs, m, p->V, ldv, p->u, p->gpart2, p->gpart, ldp, 1, p->H, p->ldh, p->ctl);
        }
    } else {
        gs_reduce(st, p->gs, p->gpart, ldp, p->H, p->ldh, p->h2, 0, p->ctl);
        {
            Prof pr(p, LP_K_GS_UPDATE, it, kk * m * 8.0 + 16.0 * m + nch * kk * 8.0 + kk * 8.0);
            gs_update(st, p->gs, m, p->V, ldv, p->u, p->h2, p->gpart, ldp, 0, p->ctl);
        }
        gs_reduce(st, p->gs, p->gpart, ldp, p->H, p->ldh, p->h2, 1, p->ctl);
        {
            Prof pr(p, LP_K_GS_UPDATE, it, kk * m * 8.0 + 16.0 * m + nch * 8.0 + kk * 8.0);
            gs_update(st, p->gs, m, p->V, ldv, p->u, p->h2, p->gpart, ldp, 1, p->ctl);
        }
    }
    gs_finish(st, p->gs, p->gpart, p->H, p->ldh, p->cs, p->sn, p->gam, p->ctl);
}

// capture `iters` Krylov iterations once per problem; every kernel argument is fixed
// (the iteration index, the done flag and the Cimmino step live in device memory), so
// the same executable graph serves every iteration of every solve
static lp_status build_graph(lp_problem* p, int iters) {
    if (!p->cap_st) LPK_HIP(hipStreamCreateWithFlags(&p->cap_st, hipStreamNonBlocking));
    hipStream_t keep = p->st;
    const uint32_t mask = p->prof_mask;
    p->prof_mask = 0;
    p->st = p->cap_st;
    hipError_t e = hipStreamBeginCapture(p->cap_st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int i = 0; i < iters; ++i) enqueue_iteration(p, -1);
        e = hipStreamEndCapture(p->cap_st, &p->graph);
    }
    p->st = keep;
    p->prof_mask = mask;
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    LPK_HIP(hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0));
    p->graph_iters = iters;
    return LP_OK;
}

lp_status krylov_solve(lp_problem* p, const double* f_dev, double tol, double* dw, double* dyh,
                       lp_krylov_info* ki) {
    hipStream_t st = p->st;
    const int64_t m = p->m, n = p->n;
    int64_t kmax = p->kmax;
    if (p->opt.krylov_max_iter > 0) kmax = std::min<int64_t>(kmax, p->opt.krylov_max_iter);
    const int64_t sid = p->solve_id++;
    if ((int64_t)p->solve_iters.size() <= sid) p->solve_iters.resize(sid + 1, 0);
    int nb = 0;
    krylov_init_rhs(st, m, f_dev, p->rho, p->fhU, p->u, p->red.part, &nb);
    krylov_init_ctl(st, m, p->red.part, nb, p->fhU, p->V, tol, (int)kmax, p->ctl, p->gam, p->omega_c);
    LPK_HIP(hipGetLastError());
    const bool use_graph = p->opt.use_graphs && p->prof_mask == 0;
    if (use_graph && !p->graph_exec) {
        lp_status grc = build_graph(p, 8);
        if (grc != LP_OK) return grc;
    }
    KrylovCtl hc;
    int64_t enq = 0;
    int batch;
    if (p->opt.poll_every > 0) batch = p->opt.poll_every;
    else batch = p->last_iters > 2 ? (int)(p->last_iters - 1) : 4;
    for (;;) {
        const int64_t todo = std::min<int64_t>(batch, kmax - enq);
        if (use_graph) {
            const int64_t launches = (todo + p->graph_iters - 1) / p->graph_iters;
            for (int64_t i = 0; i < launches; ++i) LPK_HIP(hipGraphLaunch(p->graph_exec, st));
            enq += launches * p->graph_iters;
        } else {
            for (int64_t i = 0; i < todo; ++i) enqueue_iteration(p, enq + i);
            enq += todo;
        }
        LPK_HIP(hipGetLastError());
        lp_status rc = read_ctl(p, &hc);
        if (rc != LP_OK) return rc;
        if (hc.done || enq >= kmax) break;
        if (p->opt.poll_every <= 0) batch = std::max(2, std::min(32, batch < 8 ? 4 : batch / 2));
    }
    // dyh = P y with R y = gamma; dw = A_hat^T dyh; true residual ||f_hat - A_hat dw||
    krylov_backsolve(st, p->H, p->ldh, p->gam, p->ykr, p->ctl);
    krylov_combine(st, m, p->P, p->ldv, p->ykr, dyh, p->ctl);
    spmv_f64(st, p->g_csc, (int)n, p->cp, p->ri, p->ahc, dyh, dw, EPI_PLAIN, nullptr, nullptr, nullptr);
    const int nbr = spmv_f64_nrm(st, p->g_csr, (int)m, p->rp, p->ci, p->ah, dw, p->dtmp_m, EPI_B_MINUS, p->fhU, p->spart);
    krylov_true_res(st, p->spart, nbr, p->ctl);
    LPK_HIP(hipGetLastError());
    lp_status rc = read_ctl(p, &hc);
    if (rc != LP_OK) return rc;
    if (ki) {
        ki->iters = hc.iters;
        ki->beta = hc.beta;
        ki->res_est = hc.res;
        ki->res_true = hc.res_true;
        ki->failed = hc.failed;
        ki->pad0 = 0;
    }
    p->solve_iters[sid] = hc.iters;
    if (p->prof_recs.size() > 200000) prof_collect(p);
    p->last_iters = hc.iters;
    p->krylov_total += hc.iters;
    return LP_OK;
}

}  // namespace lpk

using namespace lpk;

// ------------------------------------------------------------------------------------
// Timing replay: the launches of one kernel class, captured once with a control block at
// k = 0 and replayed back-to-back between two events on the problem's stream.
extern "C" lp_status lp_time_kernel(lp_problem* p, int32_t cls, int32_t reps, double* us_per_launch,
                                    double* bytes_per_launch, double* flops_per_launch,
                                    int32_t* launches_per_group) {
    if (!p || reps < 1 || !us_per_launch) return LP_EINVAL;
    if (!p->have_point) {
        set_error("no scaling yet: run ipm_step, lp_solve or direction_solve first");
        return LP_EINVAL;
    }
    if (cls == LP_K_GRAM && !p->gsor) {
        set_error("no dense Gram path for this problem");
        return LP_EINVAL;
    }
    if (cls != LP_K_SWEEP && cls != LP_K_SPMV_CSR && cls != LP_K_SPMV_CSC && cls != LP_K_GRAM) {
        set_error("timing replay covers the sweep, the two sparse products and the Gram build");
        return LP_EINVAL;
    }
    hipStream_t st = p->st;
    // control block for the replay: k = 0, not done, the current Cimmino step
    KrylovCtl t{};
    t.kmax = 1;
    t.omega_c = p->omega_c;
    *p->host_ctl = t;
    LPK_HIP(hipMemcpyAsync(p->tctl, p->host_ctl, sizeof(KrylovCtl), hipMemcpyHostToDevice, st));
    LPK_HIP(hipStreamSynchronize(st));
    if (!p->cap_st) LPK_HIP(hipStreamCreateWithFlags(&p->cap_st, hipStreamNonBlocking));
    const uint32_t mask = p->prof_mask;
    p->prof_mask = 0;
    double bytes = 0.0, flops = 0.0;
    int64_t launches = 0;
    p->count_bytes = &bytes;
    p->count_flops = &flops;
    p->count_launch = &launches;
    p->count_cls = cls;
    hipStream_t keep = p->st;
    p->st = p->cap_st;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(p->cap_st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const int64_t m = p->m, n = p->n, nnz = p->nnz;
        if (cls == LP_K_SWEEP) {
            enqueue_precond(p, p->tctl, -1, false);
        } else if (cls == LP_K_SPMV_CSC) {
            Prof pr(p, LP_K_SPMV_CSC, -1, nnz * 12.0 + m * 8.0 + n * 8.0 + (n + 1) * 4.0);
            spmv_f64_col(p->st, p->g_csc, (int)n, p->cp, p->ri, p->ahc, p->P, p->ldv, p->z64, p->tctl);
        } else if (cls == LP_K_SPMV_CSR) {
            if (p->gsor) {
                Prof pr(p, LP_K_SPMV_CSR, -1, 8.0 * m * m + 16.0 * m);
                gemv_col(p->st, (int)m, p->G, p->P, p->ldv, p->u, p->tctl);
            } else {
                Prof pr(p, LP_K_SPMV_CSR, -1, nnz * 12.0 + n * 8.0 + m * 8.0 + (m + 1) * 4.0);
                spmv_f64(p->st, p->g_csr, (int)m, p->rp, p->ci, p->ah, p->z64, p->u, EPI_PLAIN, nullptr, nullptr,
                         &p->tctl->done);
            }
        } else {
            (void)build_dense_preconditioner(p);
        }
        e = hipStreamEndCapture(p->cap_st, &g);
    }
    p->st = keep;
    p->prof_mask = mask;
    p->count_bytes = nullptr;
    p->count_flops = nullptr;
    p->count_launch = nullptr;
    if (e != hipSuccess) return hip_fail(e, "timing capture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "timing graph instantiate");
    }
    hipEvent_t a = nullptr, b = nullptr;
    LPK_HIP(hipEventCreate(&a));
    LPK_HIP(hipEventCreate(&b));
    LPK_HIP(hipGraphLaunch(ex, st));   // warm
    LPK_HIP(hipEventRecord(a, st));
    for (int32_t r = 0; r < reps; ++r) LPK_HIP(hipGraphLaunch(ex, st));
    LPK_HIP(hipEventRecord(b, st));
    LPK_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    LPK_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipGraphExecDestroy(ex);
    (void)hipGraphDestroy(g);
    const double per = launches > 0 ? (double)launches : 1.0;
    *us_per_launch = (double)ms * 1e3 / ((double)reps * per);
    if (bytes_per_launch) *bytes_per_launch = bytes / per;
    if (flops_per_launch) *flops_per_launch = flops / per;
    if (launches_per_group) *launches_per_group = (int32_t)launches;
    return LP_OK;
}
