// direction_solve_noalloc: the search-direction solve of direction_solve for callers that
// cannot allocate device memory during the call (code under stream capture, tight serving
// loops, harnesses that forbid allocation).  Its per-call device storage -- the batch
// descriptors, the Krylov control block, the phase parameters, the reduction partials and
// the Krylov workspace (basis V, multiplier vectors P, Hessenberg matrix H, Givens and
// Gram-Schmidt arrays) -- lives in one file-scope device array, `scratch`, of fixed size,
// which every GPU the library runs on holds until the process ends.  The kernels are those
// of direction_solve, launched one by one (no graph is instantiated).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "lpk_impl.h"

namespace lpk {

constexpr size_t SCRATCH_BYTES = (size_t)32 << 20;   // 32 MiB per device

// Host code must not pass `scratch` itself to a kernel or a copy: in host code the name
// is a host-side stand-in.  Its device address, per device, comes from
// hipGetSymbolAddress (scratch_base below).
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// the device address of `scratch` on device dev (the current device), looked up once
static lp_status scratch_base(int dev, unsigned char** out) {
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) {
        set_error("direction_solve_noalloc: device index beyond 63");
        return LP_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* q = nullptr;
        const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = (unsigned char*)q;
    }
    *out = g_scratch_ptr[dev];
    return LP_OK;
}

// The Krylov workspace of problem p, in the shapes lp_create gives it (ldv = m, ldh =
// basis columns), carved from base; returns the bytes it spans (each array 256-aligned).
struct Workspace {
    double *V, *P, *H, *cs, *sn, *gam, *ykr, *h2, *gpart, *gpart2;
};

static size_t carve_workspace(const lp_problem* p, unsigned char* base, Workspace* w) {
    const bool gmres = p->opt.krylov == LP_ABGMRES || p->opt.krylov == LP_BAGMRES;
    const int64_t cols = gmres ? p->kmax + 1 : 1;
    const int64_t pcols = p->opt.krylov == LP_ABGMRES ? p->kmax + 1 : 1;
    const int64_t segs = gs_segments(p->m);
    size_t off = 0;
    auto take = [&](int64_t count) {
        double* q = base ? (double*)(base + off) : nullptr;
        off += align256(sizeof(double) * (size_t)std::max<int64_t>(1, count));
        return q;
    };
    Workspace x;
    x.V = take(p->m * cols);
    x.P = take(p->m * pcols);
    x.H = take(cols * cols);
    x.cs = take(cols + 1);
    x.sn = take(cols + 1);
    x.gam = take(cols + 1);
    x.ykr = take(cols + 1);
    x.h2 = take(cols + 1);
    if (gmres) {
        x.gpart = take(std::max<int64_t>(p->nchunks, segs * (cols + 1)));
        x.gpart2 = take(segs * (cols + 1));
    } else {
        x.gpart = take(p->nchunks);
        x.gpart2 = nullptr;
    }
    if (w) *w = x;
    return off;
}

// points the problem's Krylov workspace (and its graph option) elsewhere for the call,
// and back when the call returns
struct WorkspaceSwap {
    lp_problem* p;
    Workspace keep;
    int32_t graphs;
    WorkspaceSwap(lp_problem* q, const Workspace& w) : p(q) {
        keep = Workspace{p->V, p->P, p->H, p->cs, p->sn, p->gam, p->ykr, p->h2, p->gpart, p->gpart2};
        graphs = p->opt.use_graphs;
        p->V = w.V; p->P = w.P; p->H = w.H; p->cs = w.cs; p->sn = w.sn; p->gam = w.gam;
        p->ykr = w.ykr; p->h2 = w.h2; p->gpart = w.gpart; p->gpart2 = w.gpart2;
        p->opt.use_graphs = 0;
    }
    ~WorkspaceSwap() {
        p->V = keep.V; p->P = keep.P; p->H = keep.H; p->cs = keep.cs; p->sn = keep.sn; p->gam = keep.gam;
        p->ykr = keep.ykr; p->h2 = keep.h2; p->gpart = keep.gpart; p->gpart2 = keep.gpart2;
        p->opt.use_graphs = graphs;
        if (p->solo) p->solo->dirty = true;   // its descriptors are rebuilt from the problem
    }
};

static lp_status bad(lp_status s, const std::string& msg) {
    set_error(msg);
    return s;
}

}  // namespace lpk

using namespace lpk;

extern "C" lp_status direction_solve_noalloc(lp_problem* p, const double* d, const double* f, double tol,
                                             double* dw, double* dy, lp_krylov_info* ki) {
    set_error("");
    if (!p) return bad(LP_EINVAL, "NULL problem");
    if (!f || !dw) return bad(LP_EINVAL, "NULL f or dw");
    if (!(tol >= 0.0)) return bad(LP_EINVAL, "tol must be >= 0");
    if (!d && !p->have_point) return bad(LP_EINVAL, "no current iterate: pass d");
    int dev = -1;
    LPK_HIP(hipGetDevice(&dev));
    if (dev != p->device) return bad(LP_EDEVICE, "direction_solve_noalloc: the problem lives on another device");
    const size_t need = BATCH_EXTERNAL_BYTES + carve_workspace(p, nullptr, nullptr);
    if (need > SCRATCH_BYTES)
        return bad(LP_ETOOBIG, "direction_solve_noalloc: m = " + std::to_string(p->m) + " with a Krylov limit of " +
                                   std::to_string(p->kmax) + " needs " + std::to_string(need) +
                                   " bytes of scratch; the limit is " + std::to_string(SCRATCH_BYTES) +
                                   " (create the problem with a smaller krylov_max_iter)");
    unsigned char* base = nullptr;
    lp_status rc = scratch_base(dev, &base);
    if (rc != LP_OK) return rc;
    const int64_t m = p->m, n = p->n;
    hipStream_t st = p->st;
    Workspace w;
    carve_workspace(p, base + BATCH_EXTERNAL_BYTES, &w);
    WorkspaceSwap swap(p, w);
    Slot hs;
    Param hp;
    Inst hic;
    Batch B;
    if ((rc = B.init_external(st, base, &hs, &hp, &hic)) != LP_OK) return rc;
    B.mem[0] = p;
    if ((rc = B.refresh()) != LP_OK) return rc;
    Param& pr = B.h_param[0];
    if (d) {
        LPK_HIP(hipMemcpyAsync(p->vec[V_D], d, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    } else {
        // D = diag(sqrt(x/s)) of the current iterate
        pr.mode = MD_RUN | MD_SCALE;
        if ((rc = B.put_params()) != LP_OK) return rc;
        b_scaling(B.L);
        LPK_HIP(hipStreamSynchronize(st));   // the parameters are written again below
    }
    pr.mode = MD_API;
    pr.scal[SC_TOL] = tol;
    if (p->opt.inner == LP_CIMMINO && !p->gsor) {
        if (p->opt.omega_c > 0.0) pr.scal[SC_OMC] = p->opt.omega_c;
        else pr.mode |= MD_POW;
    }
    if ((rc = B.put_params()) != LP_OK) return rc;
    if ((rc = scale_batch(B, MD_API)) != LP_OK) return rc;
    LPK_HIP(hipMemcpyAsync(p->vec[V_TMPM], f, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    gather(st, m, p->vec[V_TMPM], p->perm_d, p->vec[V_F]);
    std::vector<lp_krylov_info> info;
    if ((rc = krylov_batch(B, MD_API, &info)) != LP_OK) return rc;
    if (ki) *ki = info[0];
    LPK_HIP(hipMemcpyAsync(dw, p->vec[V_DW], sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    if (dy) {
        b_div_rho(B.L, V_DYC, V_DYH, MD_API);
        scatter(st, m, p->vec[V_DYC], p->perm_d, p->vec[V_TMPM]);
        LPK_HIP(hipMemcpyAsync(dy, p->vec[V_TMPM], sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    }
    LPK_HIP(hipGetLastError());
    LPK_HIP(hipStreamSynchronize(st));
    return LP_OK;
}
