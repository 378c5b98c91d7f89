// Internal launch wrappers of the HIP kernels (gfx950).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpk {

// Device-resident control block of one Krylov solve.  Every kernel of the Krylov loop
// reads the current iteration index k and the done flag from here, so one iteration is
// the same launch sequence for every k (it can be captured once and replayed).
struct KrylovCtl {
    int32_t k;          // number of basis vectors already completed (iteration index)
    int32_t done;       // 1: converged, broken down or at kmax; later kernels return early
    int32_t iters;      // iterations accepted into the least-squares solution
    int32_t failed;     // 1: tolerance not met
    int32_t kmax;
    int32_t pad;
    double beta;        // ||f_hat||
    double thresh;      // tol * beta
    double res;         // |gamma_{k+1}|
    double inv_h;       // 1 / h_{k+1,k} of the last completed iteration
    double res_true;    // ||f_hat - A_hat dw||
    double omega_c;     // Cimmino step of the current scaling
};

enum Epilogue : int {
    EPI_PLAIN = 0,      // out = sum
    EPI_B_MINUS = 1,    // out = b1 - sum
    EPI_B1_MINUS_B2 = 2,// out = b1 - sum - b2
    EPI_B_PLUS = 3,     // out = b1 + sum
};

// row-dot sparse products: out[r] = epi(sum_k val[k] * x[idx[k]]), r in [0, nrows).
// Used for CSR (A x) and for CSC stored as CSR of A^T (A^T y).  g = lanes per row.
void spmv_f64(hipStream_t st, int g, int nrows, const int32_t* ptr, const int32_t* idx,
              const double* val, const double* x, double* out, int epi, const double* b1,
              const double* b2, const int32_t* skip);
void spmv_f32(hipStream_t st, int g, int nrows, const int32_t* ptr, const int32_t* idx,
              const float* val, const float* x, float* out, int epi, const double* b1,
              const int32_t* skip);
// out = A x with x = column ctl->k of the column-major X (leading dimension ldx); skipped
// once ctl->done is set
void spmv_f64_col(hipStream_t st, int g, int nrows, const int32_t* ptr, const int32_t* idx,
                  const double* val, const double* X, int64_t ldx, double* out,
                  const KrylovCtl* ctl);
// same with the sum of squares of out accumulated into per-block partials part[nblk]
int spmv_f64_nrm(hipStream_t st, int g, int nrows, const int32_t* ptr, const int32_t* idx,
                 const double* val, const double* x, double* out, int epi, const double* b1,
                 double* part);

// one colour of a NE-SOR sweep over rows [r0, r1) of the colour-permuted row-scaled CSR
void nesor_colour_f64(hipStream_t st, int g, int r0, int r1, const int32_t* ptr,
                      const int32_t* idx, const double* val, double* z, const double* V,
                      double* P, int64_t ldv, double omega, const KrylovCtl* ctl, int write_z);
void nesor_colour_f32(hipStream_t st, int g, int r0, int r1, const int32_t* ptr,
                      const int32_t* idx, const float* val, float* z, const double* V,
                      double* P, int64_t ldv, double omega, const KrylovCtl* ctl, int write_z);

// Cimmino pieces: p_k += w * r, with r = v_k - A z (first sweep: r = v_k)
void cimmino_residual_f64(hipStream_t st, int g, int m, const int32_t* ptr, const int32_t* idx,
                          const double* val, const double* z, const double* V, double* P,
                          int64_t ldv, double omega_c, double* r, int first, const KrylovCtl* ctl);
void cimmino_residual_f32(hipStream_t st, int g, int m, const int32_t* ptr, const int32_t* idx,
                          const float* val, const float* z, const double* V, double* P,
                          int64_t ldv, double omega_c, float* r, int first, const KrylovCtl* ctl);
void cimmino_zupdate_f64(hipStream_t st, int g, int n, const int32_t* cptr, const int32_t* ridx,
                         const double* cval, const double* r, double* z, double omega_c, int first,
                         const KrylovCtl* ctl);
void cimmino_zupdate_f32(hipStream_t st, int g, int n, const int32_t* cptr, const int32_t* ridx,
                         const float* cval, const float* r, float* z, double omega_c, int first,
                         const KrylovCtl* ctl);

// start of Krylov iteration k: V[:,k] = U * inv_h (k >= 1), z = 0, P[:,k] = 0
void krylov_prep(hipStream_t st, int64_t m, int64_t n, double* V, const double* U, double* P,
                 int64_t ldv, double* z64, float* z32, const KrylovCtl* ctl);
// column k of P (FP64) -> the n-vector z64 = A_hat^T p  is done by spmv_f64 on the CSC;
// P column pointer for the current k
void copy_pcol(hipStream_t st, int64_t m, const double* P, int64_t ldv, double* out,
               const KrylovCtl* ctl);

// CGS2 on the basis V (column-major, leading dimension ldv, columns 0..k):
//   dots:  part[c * ldp + j] = sum_{i in chunk c} V[i, j] u[i],  j <= k
//   reduce: h[j] = sum_c part[c * ldp + j]   (accumulate = 1: h[j] += ...; also h2 out)
//   update: u[i] -= sum_j V[i, j] h[j];  then part2 dots (next pass) or norm partials
struct GsPlan {
    int rpl;            // rows per lane (chunk = 64 * rpl rows)
    int nchunks;
    int waves;          // waves per block
};
GsPlan gs_plan(int64_t m);
void gs_dots(hipStream_t st, const GsPlan& pl, int64_t m, const double* V, int64_t ldv,
             const double* u, double* part, int64_t ldp, const KrylovCtl* ctl);
void gs_reduce(hipStream_t st, const GsPlan& pl, const double* part, int64_t ldp, double* H,
               int64_t ldh, double* h2, int accumulate, const KrylovCtl* ctl);
// mode 0: update then dots of the updated u into part; mode 1: update then ||u||^2 partials
void gs_update(hipStream_t st, const GsPlan& pl, int64_t m, const double* V, int64_t ldv,
               double* u, const double* h, double* part, int64_t ldp, int mode,
               const KrylovCtl* ctl);
// update with the reduction of the previous pass's partials pin fused in (each block sums
// them; block 0 writes column k of H): usable while gs_fusable
bool gs_fusable(const GsPlan& pl, int64_t kmax);
void gs_update_fused(hipStream_t st, const GsPlan& pl, int64_t m, const double* V, int64_t ldv,
                     double* u, const double* pin, double* part, int64_t ldp, int mode,
                     double* H, int64_t ldh, const KrylovCtl* ctl);
// norm finish + Givens + convergence; single block
void gs_finish(hipStream_t st, const GsPlan& pl, const double* part, double* H, int64_t ldh,
               double* cs, double* sn, double* gam, KrylovCtl* ctl);

// solve setup: f_hat = f / rho, partial norms; then V[:,0] = f_hat / beta and ctl init
void krylov_init_rhs(hipStream_t st, int64_t m, const double* f, const double* rho, double* fh,
                     double* U, double* part, int* nblk_out);
void krylov_init_ctl(hipStream_t st, int64_t m, const double* part, int nblk, const double* fh,
                     double* V, double tol, int kmax, KrylovCtl* ctl, double* gam, double omega_c);
// back substitution R y = gamma(1:iters) (single block)
void krylov_backsolve(hipStream_t st, const double* H, int64_t ldh, const double* gam,
                      double* y, KrylovCtl* ctl);
// dyh = P[:, 0:iters] y
void krylov_combine(hipStream_t st, int64_t m, const double* P, int64_t ldv, const double* y,
                    double* dyh, const KrylovCtl* ctl);
void krylov_true_res(hipStream_t st, const double* part, int nblk, KrylovCtl* ctl);

// dense path: G = A A^T by FP64 MFMA (A dense row-major), u = G p_k
void gram_f64(hipStream_t st, int m, int64_t n, const double* A, int64_t lda, double* G, float* G32);
void gemv_col(hipStream_t st, int m, const double* G, const double* P, int64_t ldv, double* u,
              const KrylovCtl* ctl);

// dense GEMM D = alpha A B + beta E + F (+1 on the diagonal shifted by diag_r0 >= 0)
void gemm_f64(hipStream_t st, int M, int N, int K, double alpha, const double* A, int64_t lda,
              const double* B, int64_t ldb, double beta, const double* E, const double* F,
              int64_t lde, double* D, int64_t ldd, int diag_r0);
// X[r0:r0+b, 0:ncols] = forward substitution with I/omega + tril(G[r0:r0+b, r0:r0+b], -1)
void trsm_diag(hipStream_t st, int m, int r0, int b, const double* G, const double* R, int64_t ldr,
               double* X, double omega, int ncols);
void to_f32(hipStream_t st, int64_t len, const double* a, float* b);
// P[:,k] = C V[:,k]
void apply_c_f64(hipStream_t st, int m, const double* C, const double* V, double* P, int64_t ldv,
                 const KrylovCtl* ctl);
void apply_c_f32(hipStream_t st, int m, const float* C, const double* V, double* P, int64_t ldv,
                 const KrylovCtl* ctl);

// generic reductions: partial results per block, then a fixed-order finish
struct Red {
    double* part;       // [nq * maxblk]
    int maxblk;
    double* out;        // [nq] device
};
int red_blocks(int64_t len);
void red_finish(hipStream_t st, const Red& r, int nq, int nblk, const int* ops /*host, 0 sum 1 min*/);

// interior-point elementwise kernels (n-space unless noted)
void ipm_measures(hipStream_t st, const Red& r, int64_t m, int64_t n, const double* x,
                  const double* s, const double* c, const double* rd, const double* b,
                  const double* y, const double* rpv);
void ipm_scaling(hipStream_t st, int64_t n, const double* x, const double* s, const double* rd,
                 double* d, double* t);
void scale_rows(hipStream_t st, int g, int m, const int32_t* ptr, const int32_t* idx,
                const double* a, const double* d, double* rho, double* ah, float* ah32);
void scale_cols(hipStream_t st, int n, const int32_t* cptr, const int32_t* ridx, const double* ac,
                const double* d, const double* rho, double* ahc, float* ahc32);
void ipm_recover_af(hipStream_t st, const Red& r, int64_t n, const double* rd, const double* dw,
                    const double* d, const double* x, const double* s, double* ds, double* dx);
void ipm_mu_af(hipStream_t st, const Red& r, int64_t n, const double* x, const double* s,
               const double* dx, const double* ds, double ap, double ad);
void ipm_cc_rhs(hipStream_t st, int64_t n, const double* dxa, const double* dsa, const double* s,
                double smu, double* t);
void ipm_recover_cc(hipStream_t st, const Red& r, int64_t n, const double* dw, const double* d,
                    const double* x, const double* s, double smu, double* dxa, double* dsa);
void ipm_ratio(hipStream_t st, const Red& r, int64_t n, const double* x, const double* s,
               const double* dx, const double* ds);
void ipm_backtrack(hipStream_t st, const Red& r, int64_t n, const double* x, const double* s,
                   const double* dx, const double* ds, double ap, double ad);
void ipm_update(hipStream_t st, const Red& r, int64_t m, int64_t n, double* x, double* s,
                double* y, const double* dx, const double* ds, const double* dy, double ap,
                double ad);
// y += a * x (m-space), out = a / rho (dy from dyhat)
void axpy(hipStream_t st, int64_t len, double a, const double* x, double* y);
void div_by(hipStream_t st, int64_t len, const double* a, const double* rho, double* out);
void gather(hipStream_t st, int64_t len, const double* src, const int32_t* perm, double* dst);
void scatter(hipStream_t st, int64_t len, const double* src, const int32_t* perm, double* dst);
void fill(hipStream_t st, int64_t len, double v, double* dst);
// lambda of A_hat A_hat^T by power iteration (Cimmino step); w = A v / ||A v|| helpers
void vec_scale_by_norm(hipStream_t st, const Red& r, int64_t len, double* v, int nblk_from);
void sumsq(hipStream_t st, const Red& r, int64_t len, const double* v);
void lincomb(hipStream_t st, int64_t len, double a, const double* x, double b, const double* y,
             double* out);
// starting point: min x, min s into out[0..1]; shift x += ax, s += as with x.s, sum x,
// sum s into out[0..2]
void min2(hipStream_t st, const Red& r, int64_t n, const double* x, const double* s);
void shift2(hipStream_t st, const Red& r, int64_t n, double* x, double* s, double ax, double as);

}  // namespace lpk
