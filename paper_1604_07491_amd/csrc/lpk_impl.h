// Internal state of an lp_problem.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lpk.h"
#include "kernels.h"

namespace lpk {

void set_error(const std::string& msg);
lp_status hip_fail(hipError_t e, const char* what);

#define LPK_HIP(call)                                          \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return lpk::hip_fail(e_, #call); \
    } while (0)

// host greedy colouring (row i takes the smallest colour unused by earlier rows that
// share a column); returns the number of colours
int32_t greedy_colour(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci,
                      int32_t* colour, int32_t* perm);

// device bytes lp_create allocates for these sizes and options
uint64_t footprint(int64_t m, int64_t n, int64_t nnz, const lp_options& o);
// host validation of lp_create's inputs (no device call)
lp_status validate_inputs(int64_t m, int64_t n, int64_t nnz, const int64_t* rp, const int32_t* ci,
                          const double* val, const double* b, const double* c);

// lanes per row for a row-dot over rows of mean length len
int lanes_for(double len);

// owned device allocations of one problem
struct DevArena {
    std::vector<void*> ptrs;
    uint64_t bytes = 0;
    bool failed = false;
    template <typename T>
    T* alloc(int64_t count) {
        if (count <= 0) count = 1;
        void* p = nullptr;
        size_t b = (size_t)count * sizeof(T);
        b = (b + 255) & ~(size_t)255;
        if (hipMalloc(&p, b) != hipSuccess) {
            failed = true;
            return nullptr;
        }
        ptrs.push_back(p);
        bytes += b;
        return (T*)p;
    }
    void release() {
        for (void* p : ptrs) (void)hipFree(p);
        ptrs.clear();
        bytes = 0;
    }
};

struct Colour {
    int32_t r0, r1;     // rows [r0, r1) in the permuted order
    int g;              // lanes per row
    int64_t nnz;        // nonzeros of the colour
};

// one timed launch: events a (before) and b (after) on the problem's stream
struct ProfRec {
    int cls;
    int64_t solve;      // which Krylov solve it belongs to
    int64_t iter;       // host-side iteration index inside that solve (-1: not a loop kernel)
    double bytes;
    double flops;
    hipEvent_t a, b;
};

}  // namespace lpk

struct lp_problem {
    int64_t m = 0, n = 0, nnz = 0;
    lp_options opt{};
    hipStream_t st = nullptr;
    int device = 0;
    bool dense = false;
    bool gsor = false;                              // dense: SOR on the Gram matrix
    double* G = nullptr;                            // m x m Gram matrix A_hat A_hat^T
    double *Xinv = nullptr, *Tmat = nullptr, *Tmat2 = nullptr, *Cmat = nullptr, *Rblk = nullptr;
    const double* Capply = nullptr;                 // the preconditioner matrix C<l>
    float* C32 = nullptr;

    // host-side structure
    std::vector<int32_t> perm;        // permuted row t is original row perm[t]
    std::vector<lpk::Colour> colours;
    int g_csr = 64, g_csc = 1;

    lpk::DevArena arena;
    // structure and data (permuted rows)
    int32_t *rp = nullptr, *ci = nullptr, *cp = nullptr, *ri = nullptr, *perm_d = nullptr;
    double *a = nullptr, *ac = nullptr;            // A values, CSR and CSC
    double *ah = nullptr, *ahc = nullptr;          // A_hat values, CSR and CSC
    float *ah32 = nullptr, *ahc32 = nullptr;       // FP32 copies (mixed precision)
    double *b = nullptr, *c = nullptr;             // b permuted, c
    // iterate and interior-point vectors
    double *x = nullptr, *y = nullptr, *s = nullptr;
    double *d = nullptr, *rho = nullptr, *rpv = nullptr, *rdv = nullptr, *tn = nullptr;
    double *dxa = nullptr, *dsa = nullptr, *dya = nullptr, *dyc = nullptr;
    double *f = nullptr, *dw = nullptr, *dyh = nullptr, *dtmp_n = nullptr, *dtmp_m = nullptr;
    // Krylov workspace
    int64_t kmax = 0, ldv = 0, ldh = 0;
    double *V = nullptr, *P = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *gam = nullptr;
    double *ykr = nullptr, *fhU = nullptr, *u = nullptr, *z64 = nullptr, *pcol = nullptr, *h2 = nullptr;
    float *z32 = nullptr, *r32 = nullptr;
    double *r64 = nullptr;
    double* gpart = nullptr;                        // (nchunks) x (kmax+1) CGS partials
    double* gpart2 = nullptr;                       // second buffer for the fused passes
    bool gs_fused = false;
    // captured Krylov iterations (replayed with hipGraphLaunch)
    hipStream_t cap_st = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_iters = 0;
    double* spart = nullptr;                        // per-block partials of a CSR product
    double* dapi = nullptr;                         // D given to direction_solve
    double norm_b = 0.0, norm_c = 0.0;
    lpk::KrylovCtl* ctl = nullptr;
    lpk::GsPlan gs{};
    double omega_c = 0.0;                           // Cimmino step of the current scaling
    // reductions
    lpk::Red red{};
    double* host_out = nullptr;                     // pinned, 8 doubles
    lpk::KrylovCtl* host_ctl = nullptr;             // pinned
    // interior-point state
    bool have_point = false;
    bool scaled_for_d = false;                      // A_hat matches the current iterate
    lp_ipm_state ist{};
    std::vector<lp_iter_info> log;
    int64_t krylov_total = 0;
    int64_t last_iters = 0;                         // hint for the polling period
    // profiler
    uint32_t prof_mask = 0;
    lpk::KrylovCtl* tctl = nullptr;                 // control block of timing replays
    double* count_bytes = nullptr;                  // host-side accounting of one capture
    double* count_flops = nullptr;
    int64_t* count_launch = nullptr;
    int count_cls = -1;
    int64_t solve_id = 0;
    std::vector<lpk::ProfRec> prof_recs;
    std::vector<hipEvent_t> prof_pool;
    std::vector<int64_t> solve_iters;               // iterations of each profiled solve
    int64_t prof_launch[LP_K_COUNT] = {0};
    double prof_ms[LP_K_COUNT] = {0}, prof_bytes[LP_K_COUNT] = {0}, prof_flops[LP_K_COUNT] = {0};
};

namespace lpk {

// scale A_hat for the given device vector d (NULL: identity) -- rho, A_hat CSR/CSC
lp_status build_scaling(lp_problem* p, const double* d_dev);
// the Krylov solve of the row-scaled min-norm problem for the current A_hat:
// f (device, permuted rows) -> dw (n) and dyh (m, multipliers with dw = A_hat^T dyh)
lp_status krylov_solve(lp_problem* p, const double* f_dev, double tol, double* dw,
                       double* dyh, lp_krylov_info* ki);
lp_status ipm_init_point(lp_problem* p);
lp_status ipm_iterate(lp_problem* p, lp_iter_info* info);
lp_status ipm_evaluate(lp_problem* p, lp_iter_info* info);
lp_status sync_read(lp_problem* p, const double* dev, double* host, int count);

// profiler: bracket a launch of class cls with events when cls is enabled
struct Prof {
    lp_problem* p;
    int idx = -1;
    Prof(lp_problem* pp, int cls, int64_t iter, double bytes, double flops = 0.0);
    ~Prof();
};
lp_status prof_collect(lp_problem* p);
void prof_release(lp_problem* p);

}  // namespace lpk
