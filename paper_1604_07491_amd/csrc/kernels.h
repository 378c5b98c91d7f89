// Device-side data of the batched engine and the launch interface of its kernels (gfx950).
// Not part of the C ABI.
//
// Every kernel works on a batch of LP instances: the launch grid is (x, S) and
// blockIdx.y selects the instance descriptor Inst[blockIdx.y], which holds that instance's
// sizes and device pointers.  grid.x covers the largest instance; blocks beyond an
// instance's own range return at once.  A single LP is a batch of one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpk {

// Per-instance control block of one Krylov solve.  The loop kernels read the iteration
// index k and the done flag from here, so one iteration is the same launch sequence for
// every k and every instance (it is captured once and replayed).
struct KrylovCtl {
    int32_t k;          // basis vectors completed (iteration index)
    int32_t done;       // 1: converged, broken down, at kmax, or not taking part
    int32_t iters;      // iterations in the least-squares solution
    int32_t failed;     // 1: tolerance not met
    int32_t kmax;
    int32_t active;     // 1: this instance takes part in the current solve
    double beta;        // ||f_hat||
    double thresh;      // tol * beta
    double res;         // |gamma_{k+1}|
    double inv_h;       // 1 / h_{k+1,k} of the last completed iteration
    double res_true;    // ||f_hat - A_hat dw||
    double omega_c;     // Cimmino step of the current scaling
    // CGNE / MRNE: gamma of the current direction (CGNE g.Cg, MRNE q.q), MRNE's
    // coefficient of the next direction, and MRNE's start phase (0 until q_0 is formed)
    double cg_gamma;
    double cg_beta;
    int32_t cg_phase;
    // CGNE / MRNE least-residual iterate (the failure rule of Sec. 4.2): CG_SAVE, the
    // iterate now in dw, dyh has the least residual so far and the next step copies it to
    // V_DWB, V_DYB before updating; CG_RESTORE, the solve missed its tolerance and the
    // assembly puts the saved iterate back
    int32_t cg_save;
    double cg_best;     // least residual so far (dw_0 = 0 included)
    // AB-GMRES with the delayed second Gram-Schmidt pass: eta of the vector the next
    // iteration preconditions, and the last finish's nu and s_k for its update
    double dg_eta;
    double dg_nu;
    double dg_sk;
};
constexpr int CG_SAVE = 1, CG_RESTORE = 2;

// vectors of an instance, addressed by selector
enum VecSel : int {
    V_X = 0, V_Y, V_S, V_D, V_RHO, V_RP, V_RD, V_TN, V_DXA, V_DSA, V_DYA, V_DYC, V_F, V_DW, V_DYH,
    V_TMPM, V_TMPN, V_B, V_C, V_FH, V_U, V_Z64, V_R64,
    V_DYB, V_QM, V_PM,  // CGNE / MRNE m-vectors: least-residual dyh, multipliers of q and p
    V_Q, V_PV, V_DWB,   // CGNE / MRNE n-vectors: q, p, least-residual dw
    V_DXC, V_DSC,       // a centrality corrector's dx and ds (multiple correctors only)
    V_COUNT
};
constexpr int V_PCOL = -1;   // column ctl->k of the multiplier vectors P
constexpr int V_VCOL = -2;   // column ctl->k of the Krylov basis V

// pmask of the launches that take only the instances still iterating that have a search
// direction (every CGNE instance, MRNE instances past their start)
constexpr int PM_ITER_DIR = -1;
// pmask of the product z_k = A_hat^T p_k in the Krylov loop: the instances still iterating
// whose sweeps do not leave z_k themselves (Inst::keepz == 0)
constexpr int PM_NOKEEP = -2;
// pmask: the instances inside a solve whose one-block sweep does not also form u = A_hat z_k
// (Inst::fuse_u 0)
constexpr int PM_NOFUSE = -3;

// matrices of an instance for the row-dot products
enum MatSel : int { M_A_CSR = 0, M_A_CSC = 1, M_AH_CSR = 2, M_AH_CSC = 3 };

// per-instance role and phase (bit mask in *Inst::mode).  Every instance of a batch is in
// its own phase; one launch serves all instances whose mode has that phase's bit.
enum Mode : int {
    MD_RUN = 1,        // role: takes interior-point steps
    MD_INIT = 2,       // role: computes its starting point
    MD_BT = 8,         // phase: centrality test at the trial point (back-tracking)
    MD_API = 16,       // direction_solve / lp_set_state request
    MD_POW = 32,       // with MD_SCALE: estimate the Cimmino step
    MD_MEAS = 64,      // phase: residuals and error measure
    MD_SCALE = 128,    // phase: D, A_hat, first right-hand side
    MD_START = 256,    // a Krylov solve starts this round
    MD_FIN = 512,      // a Krylov solve is assembled this round
    MD_POST1 = 1024,   // phase: after the first solve
    MD_MUAF = 2048,    // phase: mu_af
    MD_RHS2 = 4096,    // phase: second right-hand side
    MD_POST2 = 8192,   // phase: after the second solve
    MD_SH1 = 16384,    // phase: starting point, first shift
    MD_SH2 = 32768,    // phase: starting point, second shift and minima
    MD_UPD = 65536,    // phase: the step x, y, s += alpha d
    MD_RHS3 = 131072,  // phase: a centrality corrector's right-hand side
    MD_POST3 = 262144, // phase: after a centrality corrector's solve
    MD_MCCADD = 524288 // phase: the accepted corrector joins the direction
};

// per-instance scalars of the current phase (Inst::scal)
enum Scal : int { SC_TOL = 0, SC_AP, SC_AD, SC_SMU, SC_HX, SC_HS, SC_OMC, SC_COUNT = 16 };

constexpr int RED_MAXBLK = 1024;
constexpr int RED_NQ = 8;

struct Inst {
    int32_t m, n, nnz, ncol;
    int32_t g_csr, g_csc, nchunks, gsor;
    int32_t rpl;                          // Gram-Schmidt rows per lane (chunk = 64 rpl rows)
    int32_t nbr;                          // blocks of the vector reductions (own sizes only)
    int32_t nbs;                          // blocks of the reduction over a CSR product
    int32_t zcover;                       // 1: the rows of colour 0 cover every column
    int32_t lds;                          // whole NE-SOR application in one block: 1 z in LDS,
                                          // 2 z, the row data, v_k and p_k in LDS
    int32_t nseg;                         // Gram-Schmidt dot segments of 1024 rows
    int64_t ldv, ldh, ldp, kmax;
    const int32_t *rp, *ci, *cp, *ri;     // CSR and CSC of the row-permuted A
    const int32_t *cstart, *cg;           // colour row ranges (ncol+1), lanes per row by colour
    const int32_t* ctab;                  // one-block sweep: colour table (4 ints per colour)
    const double *a, *ac;                 // A values (CSR, CSC)
    double *ah, *ahc;                     // A_hat values (CSR, CSC)
    float *ah32, *ahc32;                  // FP32 copies (mixed precision)
    double* vec[V_COUNT];
    float *z32, *r32;
    double *V, *P, *H, *cs, *sn, *gam, *ykr, *h2, *gpart, *gpart2;
    const double *G, *C;                  // dense path: Gram matrix and preconditioner matrix
    const float* C32;
    KrylovCtl* ctl;
    double* part;                         // reduction partials [RED_NQ][RED_MAXBLK]
    double* out;                          // reduction results [RED_NQ]
    double* scal;                         // phase scalars [SC_COUNT]
    int32_t* mode;                        // phase role (Mode bits)
    double omega;
    const int32_t* fpairs;                // split free variables: (x+ column, x- column) pairs
    int32_t nfpairs;                      // number of pairs (0 unless made with general bounds)
    int32_t fp32;                         // 1: the inner sweeps run in FP32 (z32, ah32)
    // row slices of the colours whose neighbouring rows touch neighbouring columns (the
    // sinks of a transportation matrix): SL_ROWS rows stored slot-major, element (slot s,
    // row r) of slice q at soff[q] + s * SL_ROWS + r; NULL cslice: no such colour
    const int32_t* cslice;                // first slice of each colour, -1: CSR rows
    const int32_t *soff, *slen;           // per slice: offset, slots (a multiple of SL_GROUPS)
    const int32_t* rsl;                   // per row: position of its slot 0, -1 if not sliced
    const int32_t* sl_idx;                // column of each sliced element, -1 for padding
    double* sl_val;                       // A_hat at the sliced elements (0 for padding)
    float* sl_val32;                      // FP32 copy (mixed precision)
    const int32_t* srows;                 // per slice: first row, rows (2 entries)
    int32_t nsl;                          // slices over all colours
    int32_t nbc;                          // blocks of the CSR rows in the product with slices
    const int32_t* crow;                  // with slices: the rows kept in CSR form only
    int32_t ncrow;                        // their number
    int32_t keepz;                        // 1: FP64 NE-SOR / NE-SSOR sweeps leave z_k = A_hat^T p_k
                                          // in V_Z64 (no product with A_hat^T in the loop)
    int32_t fuse_u;                       // 1: the one-block sweep of an AB-GMRES iteration also
                                          // forms u = A_hat z_k into V_U (no product launch)
};

#ifndef LPK_SL_GROUPS
#define LPK_SL_GROUPS 32
#endif
constexpr int SL_ROWS = 16;               // rows of a slice
constexpr int SL_GROUPS = LPK_SL_GROUPS;  // slot groups of a slice's block (4 per wave)
constexpr int SL_THREADS = SL_ROWS * SL_GROUPS;

// host-side launch description of a batch (maxima over its instances)
struct BLaunch {
    const Inst* I;          // device array of S descriptors
    int S;
    hipStream_t st;
    int max_m, max_n;
    int max_nbr, max_nbs;   // largest per-instance reduction block counts
    int64_t max_ldp;        // largest kmax + 1
    int grid_spmv[4];       // blocks of the row-dot products over each matrix
    int gs_rpl, gs_nchunks; // largest rows per lane (template bound) and chunk count
    int gs_dots_grid;       // blocks per instance of the Gram-Schmidt dot launches
    bool gs_fused;          // every update block sums the dot partials itself
    bool any32, any64;      // some instance sweeps in FP32 / in FP64 (Inst::fp32); a launch of
                            // either precision skips the instances of the other
    bool any_nokeep;        // some instance needs z_k = A_hat^T p_k from a product (Inst::keepz 0)
    bool any_fuse, all_fuse;// some / every instance forms u = A_hat z_k in its sweep (Inst::fuse_u)
    int inner;              // lp_inner of every instance (NE-SOR, Cimmino, NE-SSOR) or 3: dense SOR
    int ell;                // inner sweeps per preconditioner application
    int krylov;             // lp_krylov of every instance (0 AB-GMRES, 1 CGNE, 2 MRNE)
    int max_ncol;
    const int* grid_colour; // host array [2 max(1, max_ncol)]: blocks of each colour's CSR launch,
                            // then of its sliced launch (0: none)
    const char* colour_r;   // host array, same layout: elements (CSR) or slot steps (sliced) per
                            // lane in registers (8, 16, 32; sliced launches also 12)
    bool need_prep;         // some NE-SOR instance needs z cleared before its first sweep
    bool any_lds;           // some instance sweeps in one block with z in LDS (lds == 1)
    int lds_bytes;          // largest z of those instances
    bool any_stage;         // some instance sweeps in one block from LDS alone (lds == 2)
    int stage_bytes;        // largest LDS footprint of those instances
    bool ba;                // BA-GMRES: the sweeps map V_U to V_U (input kept in V_R64)
    bool any_free;          // some instance has split free variables
    int grid_ahz;           // blocks of u = A_hat z with slices (0: no instance has slices)
    int max_fpairs;         // most split free variables of an instance
    int max_ncol_global;    // colours of the instances swept by per-colour launches
};

// An NE-SOR / NE-SSOR instance sweeps in one block with all of its row values and column
// indices, z, v_k, p_k and the row pointers in LDS when they fit in
// LDS_STAGE_MAX (lds_stage_bytes); with all but the row values and indices in LDS when
// those fit in LDS_Z_MAX (lds_z_bytes), the rows then read from memory.  gfx950 gives a
// workgroup 160 KiB of LDS.
constexpr int LDS_BLOCK_MAX = 160 * 1024;
constexpr int LDS_Z_MAX = LDS_BLOCK_MAX;
constexpr int LDS_STAGE_MAX = LDS_BLOCK_MAX;
// LDS of the one-block sweep: z, v_k, p_k and the row pointers, and (staged) the rows too
inline int64_t lds_z_bytes(int64_t m, int64_t n, int tbytes) {
    return 16 * m + (n + 1) * tbytes + 4 * (m + 1);
}
// threads of the one-block sweep, and the most rounds of them a colour's rows may take
// when the rows are read from memory (each round is one dependent load step)
constexpr int LDS_SWEEP_THREADS = 1024;
constexpr int LDS_ROUNDS_MAX = 4;
// element slots per lane held in registers by the one-block sweep, and the most lanes it
// gives a row whose longest row fits in that many slots (colours of the one-block sweep take
// min(lanes_for(mean length), LDS_LANES_MAX) lanes a row then; measured on the serving mix:
// 16 lanes 160 us per 256-LP launch, 8 lanes 170 us, up to 64 lanes 185 us)
constexpr int LDS_SLOTS = 16;
constexpr int LDS_LANES_MAX = 16;
inline int64_t lds_stage_bytes(int64_t m, int64_t n, int64_t nnz, int tbytes) {
    return 16 * m + nnz * (tbytes + 4) + (n + 1) * tbytes + 4 * (m + 1);
}
// The one-block sweep's colour table, four ints per colour in device memory, read by
// scalar loads: first and last row, lanes per row g, and (bit 0) whether the colour runs
// on wave 0 alone (rows x g <= 64) with (bits 1..) the element slots per lane its longest
// row needs, ceil(longest / g), rounded up to a count the kernel compiles (slot_class); a
// colour needing more than LDS_SLOTS takes the element loop.
__host__ __device__ constexpr int slot_class(int slots) {
    return slots <= 4 ? slots : slots <= 6 ? 6 : slots <= 8 ? 8 : slots <= 12 ? 12 : slots <= 16 ? 16 : slots;
}

// ---- row-dot products (CSR A x, CSC A^T y) --------------------------------------------
enum Epilogue : int { EPI_PLAIN = 0, EPI_B_MINUS = 1, EPI_B1_MINUS_B2 = 2, EPI_B_PLUS = 3 };
// out = epi(sum) over the rows of matrix `mat` for every instance whose mode has a bit of
// pmask (pmask 0: instances whose Krylov solve is still running).  x = vec[xsel]
// (V_PCOL: column k of P, V_VCOL: column k of V); nrm: per-block partials of sum(out^2) into part (quantity 0,
// Inst::nbs blocks; only for the CSR matrices).
void b_spmv(const BLaunch& L, int mat, int xsel, int outsel, int epi, int b1sel, int b2sel,
            int pmask, bool nrm);

// ---- Krylov loop ------------------------------------------------------------------------
// The first sweep of every preconditioner application also writes V[:,k] = u / h_{k,k-1}
// for its rows and overwrites (rather than accumulates) p_k; b_prep only clears the NE-SOR
// z of instances whose colour 0 does not cover every column (colour 0 then overwrites z).
void b_prep(const BLaunch& L, int pmask);
// one colour of pass `pass` of `npass` (dir 0: colours in order, 1: reversed, the
// backward half of an NE-SSOR iteration); the first pass forms v_k and p_k
// pmask 0: the instances inside a solve; > 0: those whose mode has a bit of pmask (the
// start of a BA-GMRES solve applies the preconditioner to f_hat).  L.ba: the input is
// V_U unscaled, the multipliers go to V_U and the input is kept in V_R64 (V and P are
// not touched)
void b_nesor(const BLaunch& L, int colour, int pass, int npass, int dir, int pmask);
// every colour of every pass, one block per instance (ssor: passes alternate direction);
// staged: the instances with Inst::lds == 2 (row data in LDS), else those with lds == 1
void b_sweep_lds(const BLaunch& L, int npass, int ssor, int pmask, int fuse = 0);   // every LDS-resident instance
void b_cim_res(const BLaunch& L, int first);
void b_cim_z(const BLaunch& L, int first);
// classical Gram-Schmidt, pass 0 and 1: dot partials, (reduce,) update u -= V h
void b_gs_dots(const BLaunch& L, int pass);
void b_gs_reduce(const BLaunch& L, int pass);
void b_gs_update(const BLaunch& L, int pass);
void b_gs_finish(const BLaunch& L);
// AB-GMRES: Gram-Schmidt twice with the second pass delayed one iteration (kernels.hip)
void b_dgs_dots(const BLaunch& L);
void b_dgs_finish(const BLaunch& L);
void b_dgs_update(const BLaunch& L);
void b_apply_c(const BLaunch& L);       // dense: P[:,k] = C v_k

// ---- CGNE and MRNE preconditioned by inner iterations (Sec. 3.3) ------------------------
// The inner iterations act on V_U (the residual g for CGNE, A p for MRNE) and leave their
// multipliers in P[:,0]; the CSC product gives A_hat^T of those in V_Z64.  Scalars live in
// each instance's control block; every kernel returns at once for finished instances.
void b_cg_init(const BLaunch& L, int pmask);   // dw = dyh = 0, directions 0, 1/h = 1; MRNE: g = f_hat
// partials of vec[x] . y (y = vec[ys], or column 0 of P for V_PCOL) over m (nlen 0) or n
void b_cg_dot(const BLaunch& L, int xs, int ys, int nlen);
void b_cgne_dir(const BLaunch& L);     // q = A_hat^T Cg + beta q (and multipliers); q.q
void b_cgne_step(const BLaunch& L);    // alpha; dw, dyh += alpha (q, qm); g -= alpha A_hat q; g.g
void b_mrne_step(const BLaunch& L);    // start: q_0; else alpha; dw, dyh, g, q, qm updates; g.g, q.q
void b_cg_check(const BLaunch& L);     // res = ||f_hat - A_hat dw||, the stopping test, the least residual,
                                       // the next gamma (and beta)
void b_cg_restore(const BLaunch& L, int pmask);   // the least-residual iterate back after a failed solve
void b_mrne_dir(const BLaunch& L);     // p = q + beta p, pm = qm + beta pm
void b_gemv_col(const BLaunch& L);      // dense: u = G p_k
// solve set-up (instances with a bit of pmask take part; the others are marked done)
void b_init_rhs(const BLaunch& L, int pmask);
void b_init_ctl(const BLaunch& L, int pmask, int64_t kcap);   // other instances untouched
void b_backsolve(const BLaunch& L, int pmask);
void b_combine(const BLaunch& L, int pmask);   // dyh = P y (BA-GMRES: V y)

// ---- BA-GMRES (the corrector-stage remark of Sec. 3.2, eq. ba_ne): GMRES on
// C A_hat A_hat^T dyh = C f_hat in m-space, C the inner-iteration operator --------------
// start, after the preconditioner has mapped V_U = f_hat to C f_hat: beta_C = ||C f_hat||,
// gamma_0 = beta_C, threshold tol * beta_C, 1/h = 1/beta_C; done if beta_C = 0 (two launches)
void b_ba_start(const BLaunch& L, int pmask);
// V[:,k] = V_U / h_{k,k-1} for the instances still iterating: v_0 after the start, and
// the next basis vector after each Givens step (pmask 0 inside the loop)
void b_ba_vnext(const BLaunch& L, int pmask);
void b_true_res(const BLaunch& L, int pmask);

// ---- scaling (Sec. 2.2, 3.5) ------------------------------------------------------------
// MD_SCALE instances: d = sqrt(x/s), t = d^2 r_d; with MD_INIT: d = 1, t = 0
void b_scaling(const BLaunch& L);
void b_scale_rows(const BLaunch& L, int pmask);
void b_scale_cols(const BLaunch& L, int pmask);
// one step of the power iteration for the Cimmino step (step 0 starts from e / sqrt(m));
// b_set_omc then stores 1 / lambda in scal[SC_OMC]
void b_power_step(const BLaunch& L, int pmask, int step);
void b_set_omc(const BLaunch& L, int pmask);

// ---- interior-point phases --------------------------------------------------------------
// out[q] = sum (ops[q] 0) or min (1) of part[q, 0:nb], nb = Inst::nbr (which 0) or nbs (1)
void b_red_finish(const BLaunch& L, int nq, const int* ops, int pmask, int which);
// every reduction below uses Inst::nbr blocks per instance
void b_measures(const BLaunch& L, int pmask);   // q0 x.s, q1 c.x, q2 ||r_d||^2, q3 b.y, q4 ||r_p||^2
void b_post1(const BLaunch& L);           // MD_POST1: q0, q1 ratio minima (MD_RUN) / x = dw (MD_INIT)
void b_mu_af(const BLaunch& L);           // MD_MUAF: q0 sum (x + ap dx)(s + ad ds)
void b_rhs2(const BLaunch& L);            // MD_RHS2: t for the second solve
void b_post2(const BLaunch& L);           // MD_POST2: q0, q1 minima
// multiple centrality correctors: MD_RHS3 t = -r/s for the target r at the trial point
// (SC_AP, SC_AD the aspiration step lengths, SC_SMU sigma mu); MD_POST3 the corrector
// (dxc, dyc, dsc) and the ratio minima of the corrected direction (q0, q1); MD_MCCADD
// the corrector added to the direction
void b_rhs3(const BLaunch& L);
void b_post3(const BLaunch& L);
void b_mcc_add(const BLaunch& L);
void b_shift(const BLaunch& L, int pmask);     // q0 x.s, q1 sum x, q2 sum s
void b_min2(const BLaunch& L, int pmask);      // q0 min x, q1 min s
void b_backtrack(const BLaunch& L);       // MD_BT: q3 min x_i s_i, q4 x.s at the trial point
void b_update(const BLaunch& L, int q);
// split free variables (general bounds): a pair whose smaller part exceeds
// (1 + |x+ - x-|) / 2 is lowered by the excess, both parts alike (x, A x, c^T x unchanged)
void b_free_pairs(const BLaunch& L, int pmask);   // MD_UPD: q = count of entries not finite positive
void b_div_rho(const BLaunch& L, int dst, int src, int pmask);

// ---- single-instance helpers (argument marshalling of the C ABI) -------------------------
void gather(hipStream_t st, int64_t len, const double* src, const int32_t* perm, double* dst);
void scatter(hipStream_t st, int64_t len, const double* src, const int32_t* perm, double* dst);
void fill(hipStream_t st, int64_t len, double v, double* dst);

// ---- dense path (per instance, once per scaling) -----------------------------------------
// W: workspace of gram_work_doubles(m) doubles for the split-K partial tiles (NULL: no split)
void gram_f64(hipStream_t st, int m, int64_t n, const double* A, int64_t lda, double* G, float* G32, double* W);
int gram_splits(int m);
int64_t gram_work_doubles(int m);
// W: workspace of wcap doubles for split-K partial tiles (NULL: no split)
void gemm_f64(hipStream_t st, int M, int N, int K, double alpha, const double* A, int64_t lda,
              const double* B, int64_t ldb, double beta, const double* E, const double* F,
              int64_t lde, double* D, int64_t ldd, int diag_r0, double* W, int64_t wcap);
void trsm_diag(hipStream_t st, int m, int r0, int b, const double* G, const double* R, int64_t ldr,
               double* X, double omega, int ncols);
void to_f32(hipStream_t st, int64_t len, const double* a, float* b);

int red_blocks(int64_t len);
int spmv_blocks(int64_t rows, int g);   // blocks of a row-dot launch over `rows` rows
constexpr int BLOCK_THREADS = 256;

}  // namespace lpk
