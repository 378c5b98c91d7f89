// The batched engine: interior-point iterations (Sec. 2.1) of many LPs in lockstep, each
// phase one launch for the whole batch, with the search-direction solves by AB-GMRES
// (Sec. 3.2) or CGNE / MRNE (Sec. 3.3) preconditioned by inner iterations on the
// row-scaled problem (Sec. 3.5).
//
// Differences from the paper's single-LP CPU layout, all exact in exact arithmetic:
//  * flexible final step: the multiplier vectors p_k of every preconditioner application
//    are kept (P = [p_1 .. p_k]) and the solution is dw = A_hat^T (P y).  z_k = A_hat^T p_k
//    is the z the FP64 NE-SOR sweeps maintain (as in the paper's own sweep); FP32 sweeps
//    and Cimmino leave no such z and it is recomputed in FP64 from p_k, so the Arnoldi
//    relation and dw in R(A_hat^T) hold to FP64 even when the sweeps run in FP32.  The
//    multipliers also give dy = diag(rho)^-1 P y with no extra matrix-vector product.
//  * classical Gram-Schmidt applied twice in place of modified Gram-Schmidt (Sec. 3.2 uses
//    MGS); both orthogonalise to working precision, CGS2 in two reductions per pass.
//  * the Hessenberg least-squares problem is kept in QR form by Givens rotations on the
//    device; the host only polls the convergence flags every few iterations.
//
// Every reduction of an instance is partitioned by that instance's own sizes, so a
// problem's iterates are bitwise the same alone and in any batch.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>

#include "lpk_impl.h"

namespace lpk {

double now_seconds() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int gs_rpl_for(int64_t m) {
    int rpl = 1;
    while (rpl < 8 && (int64_t)64 * rpl * 1024 < m) rpl *= 2;
    return rpl;
}

int gs_segments(int64_t m) { return (int)((m + 1023) / 1024); }

bool gs_fusable(int64_t m, int64_t kmax) { return gs_segments(m) <= 4 && kmax + 1 <= 2048; }

static inline int cdiv_i(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

bool batch_compatible(const lp_problem* a, const lp_problem* b) {
    // the sweep precision is per instance (Inst::fp32): FP32 and FP64 members share a batch
    return a->opt.inner == b->opt.inner &&
           a->opt.krylov == b->opt.krylov &&
           a->gsor == b->gsor && a->opt.inner_sweeps == b->opt.inner_sweeps && a->device == b->device;
}

// ------------------------------------------------------------------------------------
// Batch

Batch::~Batch() {
    prof_release(*this);
    drop_graph();
    if (cap_st) (void)hipStreamDestroy(cap_st);
    if (external) return;   // the storage is the caller's
    if (d_inst) (void)hipFree(d_inst);
    if (d_inst_c) (void)hipFree(d_inst_c);
    if (d_pad_slot) (void)hipFree(d_pad_slot);
    if (d_pad_param) (void)hipFree(d_pad_param);
    if (d_pad_part) (void)hipFree(d_pad_part);
    if (h_inst_c) (void)hipHostFree(h_inst_c);
    if (d_slot) (void)hipFree(d_slot);
    if (d_param) (void)hipFree(d_param);
    if (d_part) (void)hipFree(d_part);
    if (h_slot) (void)hipHostFree(h_slot);
    if (h_param) (void)hipHostFree(h_param);
    if (own_stream && st) (void)hipStreamDestroy(st);
}

lp_status Batch::init(int capacity, hipStream_t stream, bool own) {
    cap = capacity;
    st = stream;
    own_stream = own;
    (void)hipGetDevice(&device);
    mem.assign((size_t)cap, nullptr);
    h_inst.assign((size_t)cap, Inst{});
    LPK_HIP(hipMalloc(&d_inst, sizeof(Inst) * cap));
    LPK_HIP(hipMalloc(&d_inst_c, sizeof(Inst) * cap));
    LPK_HIP(hipMalloc(&d_pad_slot, sizeof(Slot)));
    LPK_HIP(hipMalloc(&d_pad_param, sizeof(Param)));
    LPK_HIP(hipMalloc(&d_pad_part, sizeof(double) * RED_NQ * RED_MAXBLK));
    LPK_HIP(hipHostMalloc((void**)&h_inst_c, sizeof(Inst) * cap, hipHostMallocDefault));
    {
        Slot ps;
        Param pp;
        memset(&ps, 0, sizeof(ps));
        memset(&pp, 0, sizeof(pp));
        ps.ctl.done = 1;
        LPK_HIP(hipMemcpy(d_pad_slot, &ps, sizeof(Slot), hipMemcpyHostToDevice));
        LPK_HIP(hipMemcpy(d_pad_param, &pp, sizeof(Param), hipMemcpyHostToDevice));
    }
    LPK_HIP(hipMalloc(&d_slot, sizeof(Slot) * cap));
    LPK_HIP(hipMalloc(&d_param, sizeof(Param) * cap));
    LPK_HIP(hipMalloc(&d_part, sizeof(double) * RED_NQ * RED_MAXBLK * cap));
    LPK_HIP(hipHostMalloc((void**)&h_slot, sizeof(Slot) * cap, hipHostMallocDefault));
    LPK_HIP(hipHostMalloc((void**)&h_param, sizeof(Param) * cap, hipHostMallocDefault));
    memset(h_slot, 0, sizeof(Slot) * cap);
    memset(h_param, 0, sizeof(Param) * cap);
    for (int i = 0; i < cap; ++i) h_slot[i].ctl.done = 1;
    LPK_HIP(hipMemcpyAsync(d_slot, h_slot, sizeof(Slot) * cap, hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemcpyAsync(d_param, h_param, sizeof(Param) * cap, hipMemcpyHostToDevice, st));
    LPK_HIP(hipStreamSynchronize(st));
    dirty = true;
    return LP_OK;
}

lp_status Batch::init_external(hipStream_t stream, unsigned char* dev, Slot* hs, Param* hp, Inst* hic) {
    external = true;
    cap = 1;
    st = stream;
    own_stream = false;
    (void)hipGetDevice(&device);
    mem.assign(1, nullptr);
    h_inst.assign(1, Inst{});
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char* q = dev + off;
        off += align256(bytes);
        return q;
    };
    d_inst = (Inst*)take(sizeof(Inst));
    d_inst_c = (Inst*)take(sizeof(Inst));
    d_pad_slot = (Slot*)take(sizeof(Slot));
    d_pad_param = (Param*)take(sizeof(Param));
    d_pad_part = (double*)take(sizeof(double) * RED_NQ * RED_MAXBLK);
    d_slot = (Slot*)take(sizeof(Slot));
    d_param = (Param*)take(sizeof(Param));
    d_part = (double*)take(sizeof(double) * RED_NQ * RED_MAXBLK);
    h_slot = hs;
    h_param = hp;
    h_inst_c = hic;
    // the storage keeps an earlier call's contents: the control blocks (done = 1, as an
    // empty slot) and the parameters start afresh; the partials are written before read
    memset(h_slot, 0, sizeof(Slot));
    memset(h_param, 0, sizeof(Param));
    h_slot->ctl.done = 1;
    LPK_HIP(hipMemcpyAsync(d_pad_slot, h_slot, sizeof(Slot), hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemcpyAsync(d_pad_param, h_param, sizeof(Param), hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemcpyAsync(d_slot, h_slot, sizeof(Slot), hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemcpyAsync(d_param, h_param, sizeof(Param), hipMemcpyHostToDevice, st));
    LPK_HIP(hipStreamSynchronize(st));
    dirty = true;
    return LP_OK;
}

int Batch::free_slot() const {
    for (int i = 0; i < cap; ++i)
        if (!mem[i]) return i;
    return -1;
}

int Batch::members() const {
    int c = 0;
    for (lp_problem* p : mem) c += p != nullptr;
    return c;
}

void Batch::drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    graph_iters = 0;
    for (int i = 0; i < NARROW; ++i) {
        if (gexec_c[i]) (void)hipGraphExecDestroy(gexec_c[i]);
        if (graph_c[i]) (void)hipGraphDestroy(graph_c[i]);
        gexec_c[i] = nullptr;
        graph_c[i] = nullptr;
    }
    c_slots.clear();
    c_width = 0;
}

static Inst make_inst(Batch& B, int slot) {
    Inst in;
    memset(&in, 0, sizeof(in));
    in.ctl = &B.d_slot[slot].ctl;
    in.out = B.d_slot[slot].out;
    in.part = B.d_part + (int64_t)slot * RED_NQ * RED_MAXBLK;
    in.scal = B.d_param[slot].scal;
    in.mode = &B.d_param[slot].mode;
    const lp_problem* p = B.mem[slot];
    if (!p) return in;
    const bool mixed = p->mixed;
    in.m = (int32_t)p->m;
    in.n = (int32_t)p->n;
    in.nnz = (int32_t)p->nnz;
    const bool sor = p->opt.inner == LP_NESOR || p->opt.inner == LP_NESSOR;
    in.ncol = (p->gsor || !sor) ? 0 : (int32_t)p->colours.size();
    in.g_csr = p->g_csr;
    in.g_csc = p->g_csc;
    in.nchunks = p->nchunks;
    in.nseg = gs_segments(p->m);
    in.gsor = p->gsor ? 1 : 0;
    in.rpl = p->rpl;
    in.nbr = red_blocks(std::max(p->m, p->n));
    in.nbs = spmv_blocks(p->m, p->g_csr);
    in.zcover = p->zcover ? 1 : 0;
    in.lds = in.ncol > 0 ? p->lds_kind : 0;
    in.ldv = p->ldv;
    in.ldh = p->ldh;
    in.ldp = p->ldh + 1;   // kmax + 2 for AB-GMRES: the dots of columns 0..kmax and u . u
    in.kmax = p->kmax;
    in.rp = p->rp;
    in.ci = p->ci;
    in.cp = p->cp;
    in.ri = p->ri;
    in.cstart = p->cstart;
    in.cg = p->cg;
    in.ctab = p->ctab;
    in.cslice = p->cslice;
    in.soff = p->soff;
    in.slen = p->slen;
    in.rsl = p->rsl;
    in.sl_idx = p->sl_idx;
    in.sl_val = p->sl_val;
    in.sl_val32 = mixed ? p->sl_val32 : nullptr;
    in.srows = p->srows;
    in.nsl = p->cslice ? p->nsl : 0;
    in.crow = p->crow;
    in.ncrow = p->ncrow;
    in.nbc = (int32_t)std::min<int64_t>(RED_MAXBLK, std::max<int64_t>(1, ((int64_t)(p->cslice ? p->ncrow : p->m) * p->g_csr + SL_THREADS - 1) / SL_THREADS));
    in.a = p->a;
    in.ac = p->ac;
    in.ah = p->ah;
    in.ahc = p->ahc;
    in.ah32 = mixed ? p->ah32 : nullptr;
    in.ahc32 = (mixed && p->opt.inner == LP_CIMMINO) ? p->ahc32 : nullptr;
    for (int v = 0; v < V_COUNT; ++v) in.vec[v] = p->vec[v];
    in.z32 = p->z32;
    in.r32 = p->r32;
    in.V = p->V;
    in.P = p->P;
    in.H = p->H;
    in.cs = p->cs;
    in.sn = p->sn;
    in.gam = p->gam;
    in.ykr = p->ykr;
    in.h2 = p->h2;
    in.gpart = p->gpart;
    in.gpart2 = p->gpart2;
    in.G = p->G;
    in.C = p->Capply;
    in.C32 = p->C32;
    in.omega = p->opt.omega;
    in.fpairs = p->fpairs;
    in.nfpairs = p->nfpairs;
    in.fp32 = mixed ? 1 : 0;
    // FP64 NE-SOR / NE-SSOR sweeps leave z_k = A_hat^T p_k for the product that follows
    // (BA-GMRES has no such product: its sweeps end the iteration's operator)
    in.keepz = (!mixed && sor && !p->gsor && p->opt.krylov != LP_BAGMRES) ? 1 : 0;
    // AB-GMRES with an FP64 one-block sweep: the sweep also forms u = A_hat z_k
    in.fuse_u = (in.keepz && in.lds != 0 && p->opt.krylov == LP_ABGMRES) ? 1 : 0;
    return in;
}

static bool same_launch(const BLaunch& a, const BLaunch& b, const std::vector<int>& ca,
                        const std::vector<int>& cb) {
    if (a.S != b.S || a.max_m != b.max_m || a.max_n != b.max_n || a.max_nbr != b.max_nbr ||
        a.max_nbs != b.max_nbs || a.max_ldp != b.max_ldp || a.gs_rpl != b.gs_rpl ||
        a.gs_nchunks != b.gs_nchunks || a.gs_fused != b.gs_fused || a.gs_dots_grid != b.gs_dots_grid || a.any32 != b.any32 ||
        a.any64 != b.any64 || a.any_nokeep != b.any_nokeep || a.any_fuse != b.any_fuse || a.all_fuse != b.all_fuse ||
        a.inner != b.inner || a.ell != b.ell || a.krylov != b.krylov || a.max_ncol != b.max_ncol ||
        a.need_prep != b.need_prep ||
        a.any_lds != b.any_lds || a.lds_bytes != b.lds_bytes || a.any_stage != b.any_stage ||
        a.stage_bytes != b.stage_bytes || a.max_ncol_global != b.max_ncol_global ||
        a.grid_ahz != b.grid_ahz)
        return false;
    for (int i = 0; i < 4; ++i)
        if (a.grid_spmv[i] != b.grid_spmv[i]) return false;
    return ca == cb;
}

static bool same_launch(const Batch& B) {
    return same_launch(B.L, B.graph_L, B.grid_colour, B.graph_colour) && B.colour_r == B.graph_r;
}

lp_status Batch::refresh() {
    L = BLaunch{};
    L.S = cap;
    L.st = st;
    L.I = d_inst;
    L.max_m = L.max_n = L.max_nbr = L.max_nbs = 1;
    L.max_ldp = 1;
    for (int i = 0; i < 4; ++i) L.grid_spmv[i] = 1;
    L.gs_rpl = 1;
    L.gs_nchunks = 1;
    L.gs_dots_grid = 1;
    L.gs_fused = true;
    L.max_ncol = 0;
    L.ell = 1;
    L.need_prep = false;
    L.any_lds = false;
    L.lds_bytes = 0;
    L.any_stage = false;
    L.stage_bytes = 0;
    L.max_ncol_global = 0;
    L.any_fuse = false;
    L.all_fuse = true;
    bool first = true;
    for (int s = 0; s < cap; ++s) {
        h_inst[s] = make_inst(*this, s);
        const lp_problem* p = mem[s];
        if (!p) continue;
        const Inst& in = h_inst[s];
        if (first) {
            L.inner = p->gsor ? 3 : p->opt.inner;
            L.ell = std::max(1, (int)p->opt.inner_sweeps);
            L.krylov = p->opt.krylov;
            L.ba = L.krylov == LP_BAGMRES;
            first = false;
        }
        // the sweep precision and whether the sweeps leave z_k are per instance
        L.any32 = L.any32 || in.fp32;
        L.any64 = L.any64 || !in.fp32;
        L.any_nokeep = L.any_nokeep || !in.keepz;
        L.any_fuse = L.any_fuse || in.fuse_u;
        L.all_fuse = L.all_fuse && in.fuse_u;
        L.max_m = std::max(L.max_m, in.m);
        L.max_n = std::max(L.max_n, in.n);
        L.max_nbr = std::max(L.max_nbr, in.nbr);
        L.max_nbs = std::max(L.max_nbs, in.nbs);
        L.max_ldp = std::max<int64_t>(L.max_ldp, in.ldp);
        const int gr = cdiv_i((int64_t)in.m * in.g_csr, BLOCK_THREADS);
        const int gc = cdiv_i((int64_t)in.n * in.g_csc, BLOCK_THREADS);
        L.grid_spmv[M_A_CSR] = std::max(L.grid_spmv[M_A_CSR], gr);
        L.grid_spmv[M_AH_CSR] = std::max(L.grid_spmv[M_AH_CSR], gr);
        L.grid_spmv[M_A_CSC] = std::max(L.grid_spmv[M_A_CSC], gc);
        L.grid_spmv[M_AH_CSC] = std::max(L.grid_spmv[M_AH_CSC], gc);
        L.gs_rpl = std::max(L.gs_rpl, in.rpl);
        L.gs_nchunks = std::max(L.gs_nchunks, in.nchunks);
        L.gs_fused = L.gs_fused && gs_fusable(p->m, p->kmax);
        // dot tasks: segments x columns (or groups of 4 columns for long bases in wide
        // batches), at most 128 blocks of 4 waves per instance, 64 in batches of 64 or more
        // (the blocks beyond a short basis's tasks return at once but still cost dispatch:
        // transportation x64, 73.4 -> 74.5 LPs/s)
        const int dcap = std::min(128, std::max(64, 4096 / std::max(1, cap)));
        const int64_t dtasks = (int64_t)in.nseg * (p->kmax + 1);
        L.gs_dots_grid = std::max<int>(L.gs_dots_grid, (int)std::min<int64_t>(dcap, cdiv_i(dtasks, 4)));
        L.max_ncol = std::max(L.max_ncol, in.ncol);
        L.any_free = L.any_free || in.nfpairs > 0;
        if (in.nsl > 0) L.grid_ahz = std::max(L.grid_ahz, in.nbc + in.nsl);
        L.max_fpairs = std::max(L.max_fpairs, in.nfpairs);
        if (in.lds == 2) {
            L.any_stage = true;
            L.stage_bytes = std::max<int>(L.stage_bytes, (int)lds_stage_bytes(in.m, in.n, in.nnz, in.fp32 ? 4 : 8));
        } else if (in.lds) {
            L.any_lds = true;
            L.lds_bytes = std::max<int>(L.lds_bytes, (int)lds_z_bytes(in.m, in.n, in.fp32 ? 4 : 8));
        } else {
            L.max_ncol_global = std::max(L.max_ncol_global, in.ncol);
            L.need_prep = L.need_prep || (in.ncol > 0 && !in.zcover);
        }
    }
    // entry c: blocks and registers of colour c's CSR launch; entry max_ncol + c: of its
    // sliced launch (0 blocks: no instance has colour c in that form)
    const int nc2 = std::max(1, L.max_ncol);
    grid_colour.assign(2 * (size_t)nc2, 0);
    colour_r.assign(2 * (size_t)nc2, 8);
    for (int s = 0; s < cap; ++s) {
        const lp_problem* p = mem[s];
        if (!p || h_inst[s].ncol == 0 || h_inst[s].lds) continue;
        for (int c = 0; c < h_inst[s].ncol; ++c) {
            const Colour& cl = p->colours[c];
            if (cl.slice0 >= 0) {
                colour_r[nc2 + c] = std::max<char>(colour_r[nc2 + c], (char)cl.sR);
                grid_colour[nc2 + c] = std::max(grid_colour[nc2 + c], cl.nslice);
                continue;
            }
            const int64_t threads = cl.il ? (int64_t)cdiv_i(cl.r1 - cl.r0, cl.il) * 64 : (int64_t)(cl.r1 - cl.r0) * cl.g;
            colour_r[c] = std::max<char>(colour_r[c], (char)cl.R);
            grid_colour[c] = std::max(grid_colour[c], cdiv_i(threads, BLOCK_THREADS));
        }
    }
    L.grid_colour = grid_colour.data();
    L.colour_r = colour_r.data();
    LPK_HIP(hipMemcpyAsync(d_inst, h_inst.data(), sizeof(Inst) * cap, hipMemcpyHostToDevice, st));
    LPK_HIP(hipStreamSynchronize(st));
    c_slots.clear();   // the narrow descriptors are rebuilt from these
    // the captured iterations read every pointer from the descriptors: they stay valid
    // while the launch shapes are unchanged
    if (!same_launch(*this)) {
        drop_graph();
        graph_L = L;
        graph_colour = grid_colour;
        graph_r = colour_r;
    }
    dirty = false;
    return LP_OK;
}

lp_status Batch::put_params() {
    // the host writes h_param again only after the previous copy has completed: either a
    // get_slots (which synchronises) came in between, or we wait here
    if (param_inflight) LPK_HIP(hipStreamSynchronize(st));
    LPK_HIP(hipMemcpyAsync(d_param, h_param, sizeof(Param) * cap, hipMemcpyHostToDevice, st));
    param_inflight = true;
    return LP_OK;
}

lp_status Batch::get_slots() {
    LPK_HIP(hipMemcpyAsync(h_slot, d_slot, sizeof(Slot) * cap, hipMemcpyDeviceToHost, st));
    LPK_HIP(hipStreamSynchronize(st));
    param_inflight = false;
    return LP_OK;
}

lp_status solo_batch(lp_problem* p, Batch** out) {
    if (!p->solo) {
        std::unique_ptr<Batch> b(new Batch());
        lp_status rc = b->init(1, p->st, false);
        if (rc != LP_OK) return rc;
        b->mem[0] = p;
        p->solo = std::move(b);
    }
    Batch* b = p->solo.get();
    if (b->dirty) {
        lp_status rc = b->refresh();
        if (rc != LP_OK) return rc;
    }
    *out = b;
    return LP_OK;
}

// ------------------------------------------------------------------------------------
// algorithmic bytes of one launch, summed over the members: every input and output the
// launch must move, each once

template <typename F>
static double over_members(const Batch& B, F f) {
    double s = 0.0;
    for (const lp_problem* p : B.mem)
        if (p) s += f(p);
    return s;
}

static double sweep_bytes_dense(const Batch& B) {
    return over_members(B, [&](const lp_problem* p) { return (double)p->m * p->m * (p->mixed ? 4.0 : 8.0) + 16.0 * p->m; });
}

// the sweeps of p leave z_k = A_hat^T p_k (FP64 NE-SOR / NE-SSOR, not BA-GMRES)
static bool keeps_z(const lp_problem* p) {
    const bool sor = p->opt.inner == LP_NESOR || p->opt.inner == LP_NESSOR;
    return !p->mixed && sor && !p->gsor && p->opt.krylov != LP_BAGMRES;
}

// the one-block sweep of p's AB-GMRES iterations also forms u = A_hat z_k (Inst::fuse_u)
static bool fuses_u(const lp_problem* p) {
    return keeps_z(p) && p->lds_kind != 0 && !p->colours.empty() && p->opt.krylov == LP_ABGMRES;
}

// ------------------------------------------------------------------------------------
// Krylov iterations

// one application of the inner-iteration preconditioner to column k of V (k and the done
// flag from each instance's control block), with the start-of-iteration preparation.
// pmask > 0 (the start of a BA-GMRES solve, NE-SOR / NE-SSOR only): the instances whose
// mode has a bit of pmask, whatever their control blocks say
static void enqueue_precond(Batch& B, int64_t it, bool with_prep, int pmask = 0, int fuse = 0) {
    const BLaunch& L = B.L;
    // bytes of one A_hat value / z entry in the sweeps of p
    auto sv = [](const lp_problem* p) { return p->mixed ? 4.0 : 8.0; };
    const int ell = L.ell;
    if (with_prep && L.need_prep) b_prep(L, pmask);
    if (L.inner == 3) {
        Prof pr(&B, LP_K_SWEEP, it, sweep_bytes_dense(B));
        b_apply_c(L);
    } else if (L.inner == LP_CIMMINO) {
        for (int sw = 0; sw < ell; ++sw) {
            const int first = sw == 0;
            {
                const double by = over_members(B, [&](const lp_problem* p) {
                    const double m = p->m, nnz = p->nnz, t = sv(p);
                    return first ? m * (8.0 + t + 16.0) : nnz * (t + 4.0) + p->n * t + m * (4.0 + 8.0 + t + 16.0);
                });
                Prof pr(&B, LP_K_SWEEP, it, by);
                b_cim_res(L, first);
            }
            if (sw + 1 < ell) {
                const double by = over_members(B, [&](const lp_problem* p) {
                    const double m = p->m, n = p->n, nnz = p->nnz, t = sv(p);
                    return nnz * (t + 4.0) + m * t + n * (4.0 + t * (first ? 1.0 : 2.0));
                });
                Prof pr(&B, LP_K_SWEEP, it, by);
                b_cim_z(L, first);
            }
        }
    } else {
        // NE-SOR: ell forward passes; NE-SSOR: ell forward-backward pairs
        const bool ssor = L.inner == LP_NESSOR;
        const int npass = ssor ? 2 * ell : ell;
        // the instances whose z fits in LDS: every pass and colour in one launch
        auto lds_kind = [&](const lp_problem* p) { return p->lds_kind; };
        if (L.any_stage || L.any_lds) {
            // staged: the row data read once per application; otherwise on every pass; both:
            // row pointers, u, v_k and p_k once, z written when kept
            const double by = over_members(B, [&](const lp_problem* p) {
                const int kd = lds_kind(p);
                if (kd == 0) return 0.0;
                // with the product fused: u written, and the rows read once more unless staged
                const double fu = (fuse && fuses_u(p)) ? 8.0 * p->m + (kd == 2 ? 0.0 : p->nnz * (sv(p) + 4.0)) : 0.0;
                return (kd == 2 ? 1 : npass) * p->nnz * (sv(p) + 4.0) + (p->m + 1) * 4.0 + (double)p->m * (8.0 + 16.0) +
                       (keeps_z(p) ? 8.0 * p->n : 0.0) + fu;
            });
            Prof pr(&B, LP_K_SWEEP, it, by);
            b_sweep_lds(L, npass, ssor ? 1 : 0, pmask, fuse);
        }
        for (int sw = 0; sw < npass; ++sw) {
            const int dir = ssor ? (sw & 1) : 0;
            for (int cc = 0; cc < L.max_ncol_global; ++cc) {
                const int c = dir ? L.max_ncol_global - 1 - cc : cc;
                const double by = over_members(B, [&](const lp_problem* p) {
                    const int nc = (int)p->colours.size();
                    if (c >= nc || lds_kind(p) != 0) return 0.0;
                    const Colour& cl = p->colours[c];
                    const int wz = keeps_z(p) || !(sw + 1 == npass && c == (dir ? 0 : nc - 1));
                    return cl.nnz * (sv(p) + 4.0) + cl.nnz * sv(p) * (wz ? 2.0 : 1.0) + (double)(cl.r1 - cl.r0) * (4.0 + 8.0 + 16.0);
                });
                Prof pr(&B, LP_K_SWEEP, it, by);
                b_nesor(L, c, sw, npass, dir, pmask);
            }
        }
    }
}

static double csc_bytes(const lp_problem* p) { return p->nnz * 12.0 + p->m * 8.0 + p->n * 8.0 + (p->n + 1) * 4.0; }
static double csr_bytes(const lp_problem* p) { return p->nnz * 12.0 + p->n * 8.0 + p->m * 8.0 + (p->m + 1) * 4.0; }

// z_k = A_hat^T p_k in FP64 for the instances whose sweeps do not leave it (FP32 sweeps,
// Cimmino): a product with the CSC copy
static void enqueue_zk(Batch& B, int64_t it) {
    if (!B.L.any_nokeep) return;
    Prof pr(&B, LP_K_SPMV_CSC, it, over_members(B, [](const lp_problem* p) { return keeps_z(p) ? 0.0 : csc_bytes(p); }));
    b_spmv(B.L, M_AH_CSC, V_PCOL, V_Z64, EPI_PLAIN, -1, -1, PM_NOKEEP, false);
}

static void enqueue_products(Batch& B, int64_t it) {
    const BLaunch& L = B.L;
    if (L.inner == 3) {
        // u = A_hat A_hat^T p_k = G p_k
        Prof pr(&B, LP_K_SPMV_CSR, it, over_members(B, [](const lp_problem* p) { return 8.0 * p->m * p->m + 16.0 * p->m; }));
        b_gemv_col(L);
        return;
    }
    // outer operator in FP64: z_k = A_hat^T p_k (left by the FP64 sweeps, else by a
    // product with the CSC copy), u = A_hat z_k (formed by the one-block sweep itself for
    // the instances with Inst::fuse_u: no launch when every instance has it)
    enqueue_zk(B, it);
    if (L.all_fuse) return;
    {
        Prof pr(&B, LP_K_SPMV_CSR, it, over_members(B, [](const lp_problem* p) { return fuses_u(p) ? 0.0 : csr_bytes(p); }));
        b_spmv(L, M_AH_CSR, V_Z64, V_U, EPI_PLAIN, -1, -1, L.any_fuse ? PM_NOFUSE : 0, false);
    }
}

// Classical Gram-Schmidt twice and the Givens step, for basis index k = it (the parts
// selected by `parts`)
enum { GS_DOTS = 1, GS_UPDATES = 2, GS_FINISH = 4 };

static void enqueue_gs(Batch& B, int64_t it, int parts) {
    const BLaunch& L = B.L;
    const double kk = (double)(it + 1);
    // V once, u once, the partials (segments x (k + 1)) once
    auto dots_b = [&]() {
        return over_members(B, [&](const lp_problem* p) { return kk * p->m * 8.0 + p->m * 8.0 + gs_segments(p->m) * kk * 8.0; });
    };
    // V once, u read and written, the partials read by every chunk's block (fused)
    auto upd_b = [&]() {
        return over_members(B, [&](const lp_problem* p) {
            return kk * p->m * 8.0 + p->m * 16.0 + (L.gs_fused ? (double)p->nchunks * gs_segments(p->m) * kk * 8.0 : kk * 8.0);
        });
    };
    for (int pass = 0; pass < 2; ++pass) {
        if (parts & GS_DOTS) {
            Prof pr(&B, LP_K_GS_DOTS, it, dots_b());
            b_gs_dots(L, pass);
        }
        if (parts & GS_UPDATES) {
            if (!L.gs_fused) b_gs_reduce(L, pass);
            Prof pr(&B, LP_K_GS_UPDATE, it, upd_b());
            b_gs_update(L, pass);
        }
    }
    if (parts & GS_FINISH) b_gs_finish(L);
}

// AB-GMRES: Gram-Schmidt twice with the second pass delayed by one iteration (one pass of
// dots and one of updates over V per iteration) and the Givens step of the column the
// iteration completes
static void enqueue_dgs(Batch& B, int64_t it, int parts) {
    const BLaunch& L = B.L;
    const double kk = (double)(it + 1);
    // V once (k + 1 columns), v~_k and u once, the partials (segments x (k + 2)) once
    auto dots_b = [&]() {
        return over_members(B, [&](const lp_problem* p) {
            return kk * p->m * 8.0 + 2.0 * p->m * 8.0 + gs_segments(p->m) * (kk + 1.0) * 16.0;
        });
    };
    // V once (k columns), v~_k and u read and written, the coefficients
    auto upd_b = [&]() {
        return over_members(B, [&](const lp_problem* p) { return (kk - 1.0) * p->m * 8.0 + p->m * 32.0 + kk * 16.0; });
    };
    if (parts & GS_DOTS) {
        Prof pr(&B, LP_K_GS_DOTS, it, dots_b());
        b_dgs_dots(L);
    }
    if (parts & GS_FINISH) b_dgs_finish(L);
    if (parts & GS_UPDATES) {
        Prof pr(&B, LP_K_GS_UPDATE, it, upd_b());
        b_dgs_update(L);
    }
}

// the residual f_hat - A_hat dw of the iterate a CGNE / MRNE step just formed, recomputed
// (its squared norm as reduction partials), for the stopping test of Sec. 4.2
static void enqueue_cg_residual(Batch& B, int64_t it) {
    Prof pr(&B, LP_K_SPMV_CSR, it, over_members(B, [](const lp_problem* p) { return csr_bytes(p) + 8.0 * p->m; }));
    b_spmv(B.L, M_AH_CSR, V_DW, V_TMPM, EPI_B_MINUS, V_FH, -1, PM_ITER_DIR, true);
}

// one CGNE or MRNE iteration (Sec. 3.3): a preconditioner application (multipliers into
// column 0 of P), its product with A_hat^T in FP64, one product with A_hat, and the
// vector kernels
static void enqueue_cg_iteration(Batch& B, int64_t it) {
    const BLaunch& L = B.L;
    auto vb = [&](double per_m, double per_n) {
        return over_members(B, [&](const lp_problem* p) { return per_m * p->m + per_n * p->n; });
    };
    if (L.krylov == LP_CGNE) {
        enqueue_precond(B, it, true);   // C g (g in V_U)
        enqueue_zk(B, it);
        {
            Prof pr(&B, LP_K_CG_VEC, it, vb(16.0, 0.0));
            b_cg_dot(L, V_U, V_PCOL, 0);
        }
        {
            Prof pr(&B, LP_K_CG_VEC, it, vb(24.0, 24.0));
            b_cgne_dir(L);
        }
        {
            Prof pr(&B, LP_K_SPMV_CSR, it, over_members(B, csr_bytes));
            b_spmv(L, M_AH_CSR, V_Q, V_TMPM, EPI_PLAIN, -1, -1, 0, false);
        }
        {
            Prof pr(&B, LP_K_CG_VEC, it, vb(48.0, 24.0));
            b_cgne_step(L);
        }
        enqueue_cg_residual(B, it);
        b_cg_check(L);
    } else {
        {
            Prof pr(&B, LP_K_SPMV_CSR, it, over_members(B, csr_bytes));
            b_spmv(L, M_AH_CSR, V_PV, V_U, EPI_PLAIN, -1, -1, PM_ITER_DIR, false);   // t = A_hat p
        }
        enqueue_precond(B, it, true);   // C t (at the start: C g)
        enqueue_zk(B, it);
        {
            Prof pr(&B, LP_K_CG_VEC, it, vb(0.0, 16.0));
            b_cg_dot(L, V_Z64, V_PV, 1);
        }
        {
            Prof pr(&B, LP_K_CG_VEC, it, vb(40.0, 40.0));
            b_mrne_step(L);
        }
        enqueue_cg_residual(B, it);
        b_cg_check(L);
        {
            Prof pr(&B, LP_K_CG_VEC, it, vb(24.0, 24.0));
            b_mrne_dir(L);
        }
    }
}

// one BA-GMRES iteration (eq. ba_ne): u = C A_hat A_hat^T v_k (both products in FP64,
// then the sweeps on u in place), CGS2 and the Givens step, v_{k+1} = u / h_{k+1,k}
static void enqueue_ba_iteration(Batch& B, int64_t it) {
    const BLaunch& L = B.L;
    {
        Prof pr(&B, LP_K_SPMV_CSC, it, over_members(B, csc_bytes));
        b_spmv(L, M_AH_CSC, V_VCOL, V_Z64, EPI_PLAIN, -1, -1, 0, false);
    }
    {
        Prof pr(&B, LP_K_SPMV_CSR, it, over_members(B, csr_bytes));
        b_spmv(L, M_AH_CSR, V_Z64, V_U, EPI_PLAIN, -1, -1, 0, false);
    }
    enqueue_precond(B, it, true);
    enqueue_gs(B, it, GS_DOTS | GS_UPDATES | GS_FINISH);
    b_ba_vnext(L, 0);
}

// one Krylov iteration (every kernel returns at once for instances whose solve is done)
static void enqueue_iteration(Batch& B, int64_t it) {
    const BLaunch& L = B.L;
    if (L.ba) {
        enqueue_ba_iteration(B, it);
        return;
    }
    if (L.krylov != LP_ABGMRES) {
        enqueue_cg_iteration(B, it);
        return;
    }
    enqueue_precond(B, it, true, 0, 1);
    enqueue_products(B, it);
    // delayed CGS2 + Givens; the host iteration index equals the device one while the solve runs
    enqueue_dgs(B, it, GS_DOTS | GS_UPDATES | GS_FINISH);
}

// capture `iters` Krylov iterations for the current membership; every kernel argument is
// fixed (the iteration index, the done flags and the Cimmino steps live in device
// memory), so the same executable graph serves every iteration of every solve
static lp_status build_graph(Batch& B, int iters) {
    if (!B.cap_st) LPK_HIP(hipStreamCreateWithFlags(&B.cap_st, hipStreamNonBlocking));
    const uint32_t mask = B.prof_mask;
    B.prof_mask = 0;
    hipStream_t keep = B.L.st;
    B.L.st = B.cap_st;
    hipError_t e = hipStreamBeginCapture(B.cap_st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int i = 0; i < iters; ++i) enqueue_iteration(B, -1);
        e = hipStreamEndCapture(B.cap_st, &B.graph);
    }
    B.L.st = keep;
    B.prof_mask = mask;
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    LPK_HIP(hipGraphInstantiate(&B.gexec, B.graph, nullptr, nullptr, 0));
    B.graph_iters = iters;
    return LP_OK;
}

// capture i of the narrower graphs: the same iterations over d_inst_c, cap >> (i + 1) wide
static lp_status build_graph_narrow(Batch& B, int i) {
    if (!B.cap_st) LPK_HIP(hipStreamCreateWithFlags(&B.cap_st, hipStreamNonBlocking));
    const uint32_t mask = B.prof_mask;
    B.prof_mask = 0;
    const BLaunch keep = B.L;
    B.L.st = B.cap_st;
    B.L.S = B.cap >> (i + 1);
    B.L.I = B.d_inst_c;
    hipError_t e = hipStreamBeginCapture(B.cap_st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int it = 0; it < 8; ++it) enqueue_iteration(B, -1);
        e = hipStreamEndCapture(B.cap_st, &B.graph_c[i]);
    }
    B.L = keep;
    B.prof_mask = mask;
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    LPK_HIP(hipGraphInstantiate(&B.gexec_c[i], B.graph_c[i], nullptr, nullptr, 0));
    return LP_OK;
}

// AB-GMRES: dyh = P y with R y = gamma, BA-GMRES: dyh = V y; dw = A_hat^T dyh (CGNE and
// MRNE update dw and dyh in the iteration); the true residual ||f_hat - A_hat dw||
static void enqueue_assembly(Batch& B, int pmask) {
    const BLaunch& L = B.L;
    if (L.krylov == LP_ABGMRES || L.ba) {
        b_backsolve(L, pmask);
        b_combine(L, pmask);
        b_spmv(L, M_AH_CSC, V_DYH, V_DW, EPI_PLAIN, -1, -1, pmask, false);
    } else {
        b_cg_restore(L, pmask);
    }
    b_spmv(L, M_AH_CSR, V_DW, V_TMPM, EPI_B_MINUS, V_FH, -1, pmask, true);
    b_true_res(L, pmask);
}

// start a solve for the pmask instances (f in V_F): f_hat, beta, control blocks;
// BA-GMRES: r_0 = C f_hat and v_0 = r_0 / ||r_0||
static void enqueue_start(Batch& B, int pmask) {
    b_init_rhs(B.L, pmask);
    b_init_ctl(B.L, pmask, 0);
    if (B.L.ba) {
        enqueue_precond(B, -1, true, pmask);
        b_ba_start(B.L, pmask);
        b_ba_vnext(B.L, pmask);
    } else if (B.L.krylov != LP_ABGMRES) {
        b_cg_init(B.L, pmask);
    }
}

lp_status krylov_batch(Batch& B, int pmask, std::vector<lp_krylov_info>* info) {
    int64_t kmax_all = 0;
    int poll_every = 0;
    bool graphs = true;
    for (int s = 0; s < B.cap; ++s) {
        const lp_problem* p = B.mem[s];
        if (!p || !(B.h_param[s].mode & pmask)) continue;
        kmax_all = std::max(kmax_all, p->kmax);
        poll_every = std::max(poll_every, (int)p->opt.poll_every);
        graphs = graphs && p->opt.use_graphs;
    }
    if (info) info->assign((size_t)B.cap, lp_krylov_info{});
    if (kmax_all == 0) return LP_OK;
    // MRNE's first launch forms q_0 and takes no step, and AB-GMRES completes column k - 1
    // in iteration k (the delayed Gram-Schmidt pass): kmax steps need kmax + 1 launches
    const int64_t extra = (B.L.krylov == LP_MRNE || (B.L.krylov == LP_ABGMRES && !B.L.ba)) ? 1 : 0;
    const int64_t sid = B.solve_id++;
    B.cur_solve = sid;
    if ((int64_t)B.solve_iters.size() <= sid) B.solve_iters.resize(sid + 1, 0);
    enqueue_start(B, pmask);
    LPK_HIP(hipGetLastError());
    const bool use_graph = graphs && B.prof_mask == 0;
    if (use_graph && !B.gexec) {
        lp_status grc = build_graph(B, 8);
        if (grc != LP_OK) return grc;
    }
    int64_t enq = 0;
    int batch = poll_every > 0 ? poll_every : (B.last_iters > 2 ? (int)(B.last_iters - 1) : 4);
    for (;;) {
        const int64_t todo = std::max<int64_t>(1, std::min<int64_t>(batch, kmax_all + extra - enq));
        if (use_graph) {
            const int64_t launches = (todo + B.graph_iters - 1) / B.graph_iters;
            for (int64_t i = 0; i < launches; ++i) LPK_HIP(hipGraphLaunch(B.gexec, B.st));
            enq += launches * B.graph_iters;
        } else {
            for (int64_t i = 0; i < todo; ++i) enqueue_iteration(B, enq + i);
            enq += todo;
        }
        LPK_HIP(hipGetLastError());
        lp_status rc = B.get_slots();
        if (rc != LP_OK) return rc;
        bool all = true;
        for (int s = 0; s < B.cap; ++s)
            if (B.mem[s] && (B.h_param[s].mode & pmask) && !B.h_slot[s].ctl.done) all = false;
        if (all || enq >= kmax_all + extra) break;
        if (poll_every <= 0) batch = std::max(2, std::min(32, batch < 8 ? 4 : batch / 2));
    }
    enqueue_assembly(B, pmask);
    LPK_HIP(hipGetLastError());
    lp_status rc = B.get_slots();
    if (rc != LP_OK) return rc;
    int64_t most = 0;
    for (int s = 0; s < B.cap; ++s) {
        lp_problem* p = B.mem[s];
        if (!p || !(B.h_param[s].mode & pmask)) continue;
        const KrylovCtl& hc = B.h_slot[s].ctl;
        if (info) {
            lp_krylov_info& ki = (*info)[s];
            ki.iters = hc.iters;
            ki.beta = hc.beta;
            ki.res_est = hc.res;
            ki.res_true = hc.res_true;
            ki.failed = hc.failed;
            ki.pad0 = 0;
        }
        p->krylov_total += hc.iters;
        p->omega_c = hc.omega_c;
        most = std::max<int64_t>(most, hc.iters);
    }
    B.solve_iters[sid] = most;
    if (B.prof_recs.size() > 200000) prof_collect(B);
    B.last_iters = most;
    return LP_OK;
}

// ------------------------------------------------------------------------------------
// Scaling

// Dense path, once per scaling: G = A_hat A_hat^T (MFMA), then the inner-iteration
// preconditioner in the matrix form of Sec. 3.1/3.2, C<l> = sum_{i<l} H^i M^-1 with the SOR
// splitting M = I/omega + tril(G, -1) (unit diagonal, Sec. 3.5) and H = I - M^-1 G:
//   X = M^-1 by block forward substitution (64-row blocks: R = I - G[B, <B] X[<B, :] by
//   GEMM, then the diagonal block's substitution), C_1 = X, C_{i+1} = X + C_i - X (G C_i).
// l SOR sweeps from zero apply exactly this C to v, so each Krylov iteration needs only
// p = C v and u = G p.
lp_status build_dense_preconditioner(Batch& B, lp_problem* p) {
    hipStream_t st = B.L.st;
    const int m = (int)p->m;
    const int64_t mm = (int64_t)m * m;
    const bool mixed = p->mixed;
    const double om = p->opt.omega;
    const int ell = std::max(1, (int)p->opt.inner_sweeps);
    const double nbt = (double)((m + 63) / 64);
    double fl = 2.0 * (double)p->n * 64.0 * 64.0 * nbt * (nbt + 1.0) / 2.0;     // Gram tiles
    fl += (double)m * m * m / 3.0 * 2.0 + (ell - 1) * 4.0 * (double)m * m * m;   // M^-1 and C
    Prof pr(&B, LP_K_GRAM, -1, 8.0 * (double)m * p->n + 8.0 * mm * (3.0 + 3.0 * (ell - 1)), fl);
    gram_f64(st, m, p->n, p->ah, p->n, p->G, nullptr, p->Wgram);
    const int64_t wcap = p->Wgram ? gram_work_doubles(m) : 0;
    fill(st, mm, 0.0, p->Xinv);
    for (int r0 = 0; r0 < m; r0 += 64) {
        const int b = std::min(64, m - r0), ncols = r0 + b;
        // R = I[B, :] - G[B, 0:r0] X[0:r0, 0:ncols]   (K = 0 for the first block: R = I)
        gemm_f64(st, b, ncols, r0, -1.0, p->G + (int64_t)r0 * m, m, p->Xinv, m, 0.0, nullptr, nullptr, m,
                 p->Rblk, m, r0, p->Wgram, wcap);
        trsm_diag(st, m, r0, b, p->G, p->Rblk, m, p->Xinv, om, ncols);
    }
    const double* Ccur = p->Xinv;
    double* bufs[2] = {p->Cmat, p->Tmat2};
    for (int i = 1; i < ell; ++i) {
        double* Cn = bufs[(i - 1) & 1];
        gemm_f64(st, m, m, m, 1.0, p->G, m, Ccur, m, 0.0, nullptr, nullptr, m, p->Tmat, m, -1, p->Wgram, wcap);
        gemm_f64(st, m, m, m, -1.0, p->Xinv, m, p->Tmat, m, 1.0, p->Xinv, Ccur, m, Cn, m, -1, p->Wgram, wcap);
        Ccur = Cn;
    }
    if (p->Capply != Ccur) {
        // the descriptor holds the preconditioner's address
        p->Capply = Ccur;
        B.dirty = true;
    }
    if (mixed) to_f32(st, mm, Ccur, p->C32);
    LPK_HIP(hipGetLastError());
    return LP_OK;
}

lp_status scale_batch(Batch& B, int pmask) {
    const BLaunch& L = B.L;
    b_scale_rows(L, pmask);
    b_scale_cols(L, pmask);
    bool pow = false;
    for (int s = 0; s < B.cap; ++s) {
        lp_problem* p = B.mem[s];
        if (!p || !(B.h_param[s].mode & pmask)) continue;
        if (p->gsor) {
            lp_status rc = build_dense_preconditioner(B, p);
            if (rc != LP_OK) return rc;
        }
        pow = pow || (B.h_param[s].mode & MD_POW);
    }
    if (B.dirty) {
        lp_status rc = B.refresh();
        if (rc != LP_OK) return rc;
    }
    if (pow) {
        // 20 power iterations on A_hat A_hat^T from e / sqrt(m): lambda = ||A_hat A_hat^T v||
        for (int step = 0; step < 20; ++step) b_power_step(B.L, MD_POW, step);
        b_set_omc(B.L, MD_POW);
    }
    LPK_HIP(hipGetLastError());
    return LP_OK;
}

// ------------------------------------------------------------------------------------
// Interior-point driver: one state machine per member, one launch per phase per round

void Engine::attach(Batch* b) {
    B = b;
    mem.assign((size_t)b->cap, Member{});
    for (int s = 0; s < b->cap; ++s) mem[s].p = b->mem[s];
}

int Engine::join(lp_problem* p, bool from_point, int32_t limit_k) {
    int s = -1;
    for (int i = 0; i < B->cap; ++i)
        if (B->mem[i] == p || (!B->mem[i] && s < 0)) {
            s = i;
            if (B->mem[i] == p) break;
        }
    if (s < 0) return -1;
    if (B->mem[s] != p) {
        B->mem[s] = p;
        B->dirty = true;
    }
    if (!from_point) {
        // x, y, s are overwritten by the starting point
        p->have_point = false;
        p->ist.k = 0;
    }
    Member mb;
    mb.p = p;
    mb.init = !from_point;
    mb.state = from_point ? MEAS : SCALE;
    mb.limit_k = limit_k;
    mb.t_join = now_seconds();
    mb.k0 = p->krylov_total;
    mem[s] = mb;
    return s;
}

void Engine::leave(int s) {
    if (B->mem[s]) {
        B->mem[s] = nullptr;
        B->dirty = true;
    }
    mem[s] = Member{};
}

bool Engine::any_live() const {
    for (const Member& mb : mem)
        if (mb.state != EMPTY && mb.state != DONE) return true;
    return false;
}

static double step_from(double minratio, double eta) {
    const double a = eta * minratio;
    return a < 1.0 ? a : 1.0;
}

static void finish(Engine::Member& mb, lp_status st) {
    mb.state = Engine::DONE;
    mb.status = st;
    mb.iters = mb.p->ist.k;
    mb.t_done = now_seconds();
}

void fill_result(const Engine::Member& mb, lp_result* r) {
    memset(r, 0, sizeof(*r));
    r->status = mb.status;
    r->iters = mb.iters;
    r->gamma = mb.last.gamma;
    r->gamma_rel = mb.last.gamma_rel;
    r->pobj = mb.last.pobj;
    r->dobj = mb.last.dobj;
    r->rp_rel = mb.last.rp_rel;
    r->rd_rel = mb.last.rd_rel;
    r->gap_rel = mb.last.gap_rel;
    r->krylov_iters = mb.p->krylov_total - mb.k0;
    r->seconds = mb.t_done - mb.t_join;
}

// residuals r_p = b - A x, r_d = c - A^T y - s, the error measure (eq. errorMeasureDef) and
// the relative stopping test; the eps_in schedule of Sec. 4.2 (x0.75 while log10 Gamma in
// (-3, 1], x0.375 at or below -3, x1.5 after a failed solve, clamped).  Returns true when
// the member stops.
static bool evaluate(Engine::Member& mb, const double* q, Param& pr) {
    lp_problem* p = mb.p;
    const lp_options& o = p->opt;
    lp_iter_info& Lg = mb.L;
    Lg = lp_iter_info{};
    const double nb = p->norm_b, nc = p->norm_c;
    Lg.mu = q[0] / (double)p->n;
    Lg.rp_rel = std::sqrt(q[4]) / (nb > 1.0 ? nb : 1.0);
    Lg.rd_rel = std::sqrt(q[2]) / (nc > 1.0 ? nc : 1.0);
    Lg.pobj = q[1];
    Lg.dobj = q[3];
    Lg.gap_rel = std::fabs(q[1] - q[3]) / (std::fabs(q[1]) > 1.0 ? std::fabs(q[1]) : 1.0);
    Lg.gamma = std::max(Lg.mu, std::max(Lg.rp_rel, Lg.rd_rel));
    Lg.gamma_rel = std::max(Lg.gap_rel, std::max(Lg.rp_rel, Lg.rd_rel));
    if (!std::isfinite(Lg.gamma_rel)) {
        set_error("non-finite residuals");
        p->log.push_back(Lg);
        mb.last = Lg;
        finish(mb, LP_DIVERGED);
        return true;
    }
    if (Lg.gamma_rel <= o.eps_out) {
        Lg.converged = 1;
        p->log.push_back(Lg);
        mb.last = Lg;
        finish(mb, LP_OK);
        return true;
    }
    if (p->ist.k >= mb.limit_k) {
        // the final point is only evaluated
        p->log.push_back(Lg);
        mb.last = Lg;
        finish(mb, LP_NOT_CONVERGED);
        return true;
    }
    if (p->ist.k >= 1) {
        const double lg = std::log10(Lg.gamma);
        double fac = 1.0;
        if (lg <= -3.0) fac = 0.375;
        else if (lg <= 1.0) fac = 0.75;
        if (p->ist.fail_prev) fac *= 1.5;
        p->ist.eps_in *= fac;
    }
    p->ist.eps_in = std::min(std::max(p->ist.eps_in, o.eps_in_min), o.eps_in_max);
    Lg.eps_in = p->ist.eps_in;
    pr.scal[SC_TOL] = p->ist.eps_in;
    return false;
}

static void take_solve(Batch& b, int s, Engine::Member& mb, lp_krylov_info* ki) {
    const KrylovCtl& hc = b.h_slot[s].ctl;
    ki->iters = hc.iters;
    ki->beta = hc.beta;
    ki->res_est = hc.res;
    ki->res_true = hc.res_true;
    ki->failed = hc.failed;
    ki->pad0 = 0;
    mb.p->krylov_total += hc.iters;
    mb.p->omega_c = hc.omega_c;
    mb.last_k = hc.iters;
    b.last_iters = hc.iters;
    if (mb.solve_id >= 0 && mb.solve_id < (int64_t)b.solve_iters.size()) b.solve_iters[mb.solve_id] = hc.iters;
}

// inside a Krylov solve; inside one or starting one this round
static bool in_krylov(Engine::State st) { return st == Engine::KRY1 || st == Engine::KRY2 || st == Engine::KRY3; }
static bool solve_phase(Engine::State st) {
    return in_krylov(st) || st == Engine::SCALE || st == Engine::RHS2 || st == Engine::RHS3;
}

// back-tracking from the current step lengths (Sec. 2.1)
static void begin_bt(Engine::Member& mb, Param& pr) {
    mb.bt = 0;
    pr.scal[SC_AP] = mb.ap;
    pr.scal[SC_AD] = mb.ad;
    mb.state = Engine::BT;
}

// Multiple centrality correctors (Gondzio): aspiration step lengths MCC_DELTA longer than
// the current ones; a corrector is kept when the shorter step length grows by at least
// MCC_GAMMA MCC_DELTA, and the sequence stops at the first miss, after max_correctors, or
// once both step lengths are 1.
constexpr double MCC_DELTA = 0.1, MCC_GAMMA = 0.1;

// the next corrector if one is due, else back-tracking
static void next_corrector(Engine::Member& mb, Param& pr, const lp_options& o) {
    if (mb.mcc < o.max_correctors && !(mb.ap >= 1.0 && mb.ad >= 1.0)) {
        pr.scal[SC_AP] = std::min(1.0, mb.ap + MCC_DELTA);
        pr.scal[SC_AD] = std::min(1.0, mb.ad + MCC_DELTA);
        mb.state = Engine::RHS3;
        return;
    }
    begin_bt(mb, pr);
}

lp_status Engine::round() {
    const lp_status rc = issue();
    if (rc != LP_OK) return rc;
    return complete();
}

bool Engine::ready() const { return !issued || hipStreamQuery(B->st) != hipErrorNotReady; }

lp_status Engine::issue() {
    Batch& b = *B;
    lp_status rc;
    if (issued) return LP_OK;
#define LPK_RC(x)                         \
    do {                                  \
        if ((rc = (x)) != LP_OK) {        \
            error = rc;                   \
            return rc;                    \
        }                                 \
    } while (0)
    if (b.dirty) LPK_RC(b.refresh());
    // Scheduling.  Members with one sparsity structure (equal m, n and nnz: the same model
    // with other data, as the LPs of one transportation network with other costs) have
    // similar solve lengths: they pass their phases together, once none of them is inside
    // a solve (lockstep; a phase costs one round for all).  Otherwise each member advances
    // as soon as its own solve ends, so no LP waits for a slower one.  Measured on 64
    // transportation LPs (lockstep faster) and on 64 random sparse LPs of one shape whose
    // solve lengths differ (advancing alone faster).
    // The options' schedule overrides the rule (2 over 1 over 0).
    int iterating = 0, sched = 0;
    bool uniform = true;
    const lp_problem* ref = nullptr;
    for (int s = 0; s < b.cap; ++s) {
        const Member& mb = mem[s];
        if (mb.state == EMPTY || mb.state == DONE) continue;
        if (in_krylov(mb.state)) ++iterating;
        sched = std::max(sched, (int)mb.p->opt.schedule);
        if (!ref) ref = mb.p;
        else if (mb.p->m != ref->m || mb.p->n != ref->n || mb.p->nnz != ref->nnz) uniform = false;
    }
    if (sched == 1) uniform = true;
    if (sched == 2) uniform = false;
    hold = uniform && iterating > 0;   // phases wait for the others' solves
    bool has[ST_COUNT] = {false};
    bool has_add = false;
    int live = 0, solving = 0, waiting = 0;
    for (int s = 0; s < b.cap; ++s) {
        Member& mb = mem[s];
        Param& pr = b.h_param[s];
        const int role = mb.init ? MD_INIT : MD_RUN;
        int md = 0;
        if (hold && mb.state != EMPTY && mb.state != DONE && !in_krylov(mb.state)) {
            pr.mode = role;
            ++live;
            continue;
        }
        switch (mb.state) {
            case MEAS: md = role | MD_MEAS; break;
            case SCALE: {
                md = role | MD_SCALE | MD_START;
                const lp_options& o = mb.p->opt;
                if (mb.init) pr.scal[SC_TOL] = o.init_tol;
                if (o.inner == LP_CIMMINO && !mb.p->gsor) {
                    if (o.omega_c > 0.0) pr.scal[SC_OMC] = o.omega_c;
                    else md |= MD_POW;
                }
                break;
            }
            case KRY1: case KRY2: case KRY3: md = role; break;
            case RHS3: md = role | MD_RHS3 | MD_START; break;
            case FIN3: md = role | MD_FIN | MD_POST3; break;
            case FIN1: md = role | MD_FIN | MD_POST1; break;
            case MUAF: md = role | MD_MUAF; break;
            case RHS2: md = role | MD_RHS2 | MD_START; break;
            case FIN2: md = role | MD_FIN | MD_POST2; break;
            case BT: md = role | MD_BT; break;
            case UPD: md = role | MD_UPD | (stepwise ? 0 : MD_MEAS); break;
            case SH1: md = role | MD_SH1; break;
            case SH2: md = role | MD_SH2; break;
            default: md = 0;
        }
        if (mb.mcc_add && mb.state != EMPTY && mb.state != DONE) {
            // an accepted corrector joins the direction this round, before the phase's kernels
            md |= MD_MCCADD;
            has_add = true;
            mb.mcc_add = false;
        }
        pr.mode = md;
        if (mb.state == EMPTY || mb.state == DONE) continue;
        has[mb.state] = true;
        ++live;
        if (solve_phase(mb.state)) ++solving;
        else ++waiting;
    }
    if (!live) return LP_OK;
    LPK_RC(b.put_params());

    // the step, then the measures of the new point (one reduction pass for both)
    const bool meas = has[MEAS] || (has[UPD] && !stepwise);
    if (has[UPD]) {
        b_update(b.L, 5);
        b_free_pairs(b.L, MD_UPD);
    }
    if (meas) {
        b_spmv(b.L, M_A_CSR, V_X, V_RP, EPI_B_MINUS, V_B, -1, MD_MEAS, false);
        b_spmv(b.L, M_A_CSC, V_Y, V_RD, EPI_B1_MINUS_B2, V_C, V_S, MD_MEAS, false);
        b_measures(b.L, MD_MEAS);
    }
    if (meas || has[UPD]) {
        const int ops[6] = {0, 0, 0, 0, 0, 0};
        b_red_finish(b.L, 6, ops, MD_MEAS | MD_UPD, 0);
    }
    // solves that finished: assembly, then direction recovery / starting-point pieces
    if (has[FIN1] || has[FIN2] || has[FIN3]) enqueue_assembly(b, MD_FIN);
    if (has[FIN1]) {
        b_post1(b.L);
        const int ops[2] = {1, 1};
        b_red_finish(b.L, 2, ops, MD_POST1, 0);
    }
    if (has[FIN2]) {
        b_post2(b.L);
        const int ops[2] = {1, 1};
        b_red_finish(b.L, 2, ops, MD_POST2, 0);
    }
    if (has[FIN3]) {
        b_post3(b.L);
        const int ops[2] = {1, 1};
        b_red_finish(b.L, 2, ops, MD_POST3, 0);
    }
    if (has[MUAF]) {
        b_mu_af(b.L);
        const int ops[1] = {0};
        b_red_finish(b.L, 1, ops, MD_MUAF, 0);
    }
    if (has_add) b_mcc_add(b.L);
    if (has[BT]) {
        b_backtrack(b.L);
        const int ops[5] = {0, 0, 0, 1, 0};
        b_red_finish(b.L, 5, ops, MD_BT, 0);
    }
    if (has[SH1] || has[SH2]) b_shift(b.L, MD_SH1 | MD_SH2);
    if (has[SH2]) b_free_pairs(b.L, MD_SH2);   // the starting point is complete
    if (has[SH2]) b_min2(b.L, MD_SH2);
    if (has[SH1]) {
        const int ops[3] = {0, 0, 0};
        b_red_finish(b.L, 3, ops, MD_SH1, 0);
    }
    if (has[SH2]) {
        const int ops[2] = {1, 1};
        b_red_finish(b.L, 2, ops, MD_SH2, 0);
    }
    // solves that start: D and A_hat, right-hand sides (predictor f = b + A (d^2 o r_d),
    // starting point f = b; corrector f = A ((dx_af o ds_af - sigma mu) / s), starting
    // point f = A c), then f_hat and the control blocks
    if (has[SCALE]) {
        b_scaling(b.L);
        LPK_RC(scale_batch(b, MD_SCALE));
        b_spmv(b.L, M_A_CSR, V_TN, V_F, EPI_B_PLUS, V_B, -1, MD_SCALE, false);
    }
    if (has[RHS2]) {
        b_rhs2(b.L);
        b_spmv(b.L, M_A_CSR, V_TN, V_F, EPI_PLAIN, -1, -1, MD_RHS2, false);
    }
    if (has[RHS3]) {   // (after the pending corrector was added above)
        b_rhs3(b.L);
        b_spmv(b.L, M_A_CSR, V_TN, V_F, EPI_PLAIN, -1, -1, MD_RHS3, false);
    }
    if (has[SCALE] || has[RHS2] || has[RHS3]) {
        enqueue_start(b, MD_START);
        for (int s = 0; s < b.cap; ++s)
            if (mem[s].state == SCALE || mem[s].state == RHS2 || mem[s].state == RHS3) {
                mem[s].solve_id = b.solve_id++;
                b.cur_solve = mem[s].solve_id;
                mem[s].enq = 0;
                if ((int64_t)b.solve_iters.size() <= mem[s].solve_id) b.solve_iters.resize(mem[s].solve_id + 1, 0);
            }
    }
    LPK_HIP(hipGetLastError());
    // Krylov iterations for every member inside a solve (the others' kernels return at
    // once): one graph of iterations while some member waits for its next phase, else
    // enough to reach the earliest expected convergence
    if (solving) {
        int64_t todo = 8;
        bool graphs = b.prof_mask == 0;
        for (int s = 0; s < b.cap; ++s)
            if (b.mem[s] && !b.mem[s]->opt.use_graphs) graphs = false;
        if (!waiting) {
            // expected iterations to the next useful poll: the first member to finish, or
            // (held phases) the last one; a member's previous solve length is the guess
            std::vector<int64_t> rs;
            for (int s = 0; s < b.cap; ++s) {
                const Member& mb = mem[s];
                if (!solve_phase(mb.state)) continue;
                const int64_t k = in_krylov(mb.state) ? b.h_slot[s].ctl.iters : 0;
                const int64_t guess = mb.last_k > 0 ? mb.last_k : b.last_iters;
                rs.push_back(std::max<int64_t>(1, guess - k));
            }
            std::sort(rs.begin(), rs.end());
            int64_t rem = rs.empty() ? 8 : rs.front();
            if (hold && !rs.empty()) {
                // the last one; with graphs, the one whose end leaves few enough members
                // iterating for the next narrower capture
                size_t idx = rs.size() - 1;
                if (graphs)
                    for (int i = 0; i < Batch::NARROW; ++i) {
                        const int w = b.cap >> (i + 1);
                        if (w >= 8 && w % 8 == 0 && (int)rs.size() > w) {
                            idx = rs.size() - (size_t)w - 1;
                            break;
                        }
                    }
                rem = rs[idx];
            }
            todo = std::max<int64_t>(8, std::min<int64_t>(rem, 256));
        }
        if (graphs && !b.gexec) LPK_RC(build_graph(b, 8));
        if (graphs) {
            // when the members inside a solve fit a narrower capture, launch that one over
            // their descriptors: the blocks of the others are never started
            std::vector<int> act;
            for (int s = 0; s < b.cap; ++s)
                if (b.mem[s] && solve_phase(mem[s].state)) act.push_back(s);
            int wi = -1;
            for (int i = Batch::NARROW - 1; i >= 0; --i) {
                const int w = b.cap >> (i + 1);
                if (w >= 8 && w % 8 == 0 && (int)act.size() <= w) {
                    wi = i;
                    break;
                }
            }
            hipGraphExec_t ex = b.gexec;
            if (wi >= 0) {
                if (!b.gexec_c[wi]) LPK_RC(build_graph_narrow(b, wi));
                const int w = b.cap >> (wi + 1);
                if (act != b.c_slots || w != b.c_width) {
                    // padding: an empty slot's descriptor over storage of its own
                    Inst pad;
                    memset(&pad, 0, sizeof(pad));
                    pad.ctl = &b.d_pad_slot->ctl;
                    pad.out = b.d_pad_slot->out;
                    pad.part = b.d_pad_part;
                    pad.scal = b.d_pad_param->scal;
                    pad.mode = &b.d_pad_param->mode;
                    for (int q = 0; q < w; ++q) b.h_inst_c[q] = q < (int)act.size() ? b.h_inst[act[q]] : pad;
                    LPK_HIP(hipMemcpyAsync(b.d_inst_c, b.h_inst_c, sizeof(Inst) * w, hipMemcpyHostToDevice, b.st));
                    b.c_slots = act;
                    b.c_width = w;
                }
                ex = b.gexec_c[wi];
            }
            const int64_t launches = (todo + b.graph_iters - 1) / b.graph_iters;
            for (int64_t i = 0; i < launches; ++i) LPK_HIP(hipGraphLaunch(ex, b.st));
            todo = launches * b.graph_iters;
        } else {
            // iteration index for the profiler (meaningful for a batch of one)
            int64_t it0 = b.cap == 1 ? mem[0].enq : -1;
            for (int64_t i = 0; i < todo; ++i) enqueue_iteration(b, it0 < 0 ? -1 : it0 + i);
        }
        for (Member& mb : mem)
            if (solve_phase(mb.state)) mb.enq += todo;
        LPK_HIP(hipGetLastError());
    }
    // the control words and reduction results come back with the round's work; the host
    // state machines advance in complete()
    LPK_HIP(hipMemcpyAsync(b.h_slot, b.d_slot, sizeof(Slot) * b.cap, hipMemcpyDeviceToHost, b.st));
    issued = true;
#undef LPK_RC
    return LP_OK;
}

lp_status Engine::complete() {
    Batch& b = *B;
    if (!issued) return LP_OK;
    issued = false;
    {
        const hipError_t e = hipStreamSynchronize(b.st);
        if (e != hipSuccess) {
            error = LP_EDEVICE;
            return hip_fail(e, "hipStreamSynchronize");
        }
    }
    b.param_inflight = false;

    // transitions (held members keep their state)
    for (int s = 0; s < b.cap; ++s) {
        Member& mb = mem[s];
        if (mb.state == EMPTY || mb.state == DONE) continue;
        if (hold && !in_krylov(mb.state)) continue;
        lp_problem* p = mb.p;
        const lp_options& o = p->opt;
        Param& pr = b.h_param[s];
        const double* q = b.h_slot[s].out;
        const bool done = b.h_slot[s].ctl.done != 0;
        switch (mb.state) {
            case UPD: {
                lp_iter_info& Lg = mb.L;
                Lg.alpha_p = mb.ap;
                Lg.alpha_d = mb.ad;
                Lg.backtracks = mb.bt;
                p->ist.fail_prev = (Lg.fail_af || Lg.fail_cc) ? 1 : 0;
                p->ist.k += 1;
                p->log.push_back(Lg);
                mb.last = Lg;
                mb.steps += 1;
                if (q[5] > 0.0) {
                    set_error("iterate left the positive orthant or became non-finite");
                    finish(mb, LP_DIVERGED);
                    break;
                }
                if (stepwise) {
                    mb.state = MEAS;
                    break;
                }
                if (!evaluate(mb, q, pr)) mb.state = SCALE;
                break;
            }
            case MEAS:
                if (!evaluate(mb, q, pr)) mb.state = SCALE;
                break;
            case SCALE:
                mb.state = done ? FIN1 : KRY1;
                break;
            case KRY1:
                if (done) mb.state = FIN1;
                break;
            case FIN1: {
                lp_krylov_info ki;
                take_solve(b, s, mb, &ki);
                if (mb.init) {
                    mb.state = RHS2;   // x~ = dw; next: f = A c
                    break;
                }
                lp_iter_info& Lg = mb.L;
                Lg.k_af = ki.iters;
                Lg.res_af = ki.beta > 0.0 ? ki.res_true / ki.beta : 0.0;
                Lg.fail_af = ki.failed;
                mb.ap = step_from(q[0], o.eta);
                mb.ad = step_from(q[1], o.eta);
                mb.cc = mb.ap < 1.0 || mb.ad < 1.0;
                if (mb.cc) {
                    pr.scal[SC_AP] = mb.ap;
                    pr.scal[SC_AD] = mb.ad;
                    mb.state = MUAF;
                } else {
                    Lg.sigma = 0.0;
                    begin_bt(mb, pr);
                }
                break;
            }
            case MUAF: {
                lp_iter_info& Lg = mb.L;
                const double mu_af = q[0] / (double)p->n;
                double sigma;
                if (Lg.gamma > 1e-3) {
                    const double r = mu_af / Lg.mu;
                    sigma = r * r;
                } else {
                    sigma = 10.0 * Lg.gamma;
                }
                if (sigma > o.sigma_max) sigma = o.sigma_max;
                Lg.sigma = sigma;
                pr.scal[SC_SMU] = sigma * Lg.mu;
                mb.state = RHS2;
                break;
            }
            case RHS2:
                mb.state = done ? FIN2 : KRY2;
                break;
            case KRY2:
                if (done) mb.state = FIN2;
                break;
            case FIN2: {
                lp_krylov_info ki;
                take_solve(b, s, mb, &ki);
                if (mb.init) {
                    // shift x~, s~ to positive (Mehrotra's heuristic)
                    pr.scal[SC_HX] = -1.5 * q[0] > 0.0 ? -1.5 * q[0] : 0.0;
                    pr.scal[SC_HS] = -1.5 * q[1] > 0.0 ? -1.5 * q[1] : 0.0;
                    mb.state = SH1;
                    break;
                }
                lp_iter_info& Lg = mb.L;
                Lg.k_cc = ki.iters;
                Lg.res_cc = ki.beta > 0.0 ? ki.res_true / ki.beta : 0.0;
                Lg.fail_cc = ki.failed;
                mb.ap = step_from(q[0], o.eta);
                mb.ad = step_from(q[1], o.eta);
                mb.mcc = 0;
                if (Lg.sigma > 0.0) next_corrector(mb, pr, o);
                else begin_bt(mb, pr);
                break;
            }
            case RHS3:
                mb.state = done ? FIN3 : KRY3;
                break;
            case KRY3:
                if (done) mb.state = FIN3;
                break;
            case FIN3: {
                lp_krylov_info ki;
                take_solve(b, s, mb, &ki);
                lp_iter_info& Lg = mb.L;
                Lg.k_mcc += ki.iters;
                mb.mcc += 1;
                const double ap2 = step_from(q[0], o.eta), ad2 = step_from(q[1], o.eta);
                if (std::min(ap2, ad2) < std::min(mb.ap, mb.ad) + MCC_GAMMA * MCC_DELTA) {
                    begin_bt(mb, pr);   // rejected: the direction stays as it was
                    break;
                }
                mb.ap = ap2;
                mb.ad = ad2;
                mb.mcc_add = true;
                Lg.correctors += 1;
                next_corrector(mb, pr, o);
                break;
            }
            case BT:
                if (q[3] >= o.phi * q[4] / (double)p->n || mb.bt >= o.max_backtrack) {
                    pr.scal[SC_AP] = mb.ap;
                    pr.scal[SC_AD] = mb.ad;
                    mb.state = UPD;
                } else {
                    mb.ap *= o.backtrack;
                    mb.ad *= o.backtrack;
                    mb.bt += 1;
                    pr.scal[SC_AP] = mb.ap;
                    pr.scal[SC_AD] = mb.ad;
                }
                break;
            case SH1:
                // balance: x += 1/2 x^T s / sum(s), s += 1/2 x^T s / sum(x)
                pr.scal[SC_HX] = 0.5 * q[0] / q[2];
                pr.scal[SC_HS] = 0.5 * q[0] / q[1];
                mb.state = SH2;
                break;
            case SH2:
                if (!(q[0] > 0.0) || !(q[1] > 0.0)) {
                    set_error("starting point is not strictly positive");
                    finish(mb, LP_DIVERGED);
                } else {
                    p->have_point = true;
                    p->ist.eps_in = o.eps_in0;
                    p->ist.k = 0;
                    p->ist.fail_prev = 0;
                    mb.init = false;
                    mb.state = MEAS;
                }
                break;
            default:
                break;
        }
    }
    if (b.prof_recs.size() > 200000) prof_collect(b);
    return LP_OK;
}

}  // namespace lpk

using namespace lpk;

lp_problem::~lp_problem() {
    solo.reset();
    arena.release();
}

// ------------------------------------------------------------------------------------
// Timing replay: the launches of one kernel class for every member of a batch, captured
// once with control blocks at k = 0 and replayed back-to-back between two events on the
// batch's stream.
static lp_status time_kernel(Batch& B, int32_t cls, int32_t reps, double* us_per_launch,
                             double* bytes_per_launch, double* flops_per_launch, int32_t* launches_per_group) {
    if (reps < 1 || !us_per_launch) return LP_EINVAL;
    if (cls != LP_K_SWEEP && cls != LP_K_SPMV_CSR && cls != LP_K_SPMV_CSC && cls != LP_K_GRAM &&
        cls != LP_K_GS_DOTS && cls != LP_K_GS_UPDATE) {
        set_error("timing replay covers the sweep, the sparse products, Gram-Schmidt and the Gram build");
        return LP_EINVAL;
    }
    const bool gs = cls == LP_K_GS_DOTS || cls == LP_K_GS_UPDATE;
    int64_t kg = 127;   // Gram-Schmidt classes: basis of kg + 1 vectors
    for (int s = 0; s < B.cap; ++s) {
        lp_problem* p = B.mem[s];
        if (!p) continue;
        if (!p->have_point && p->krylov_total == 0) {
            set_error("no scaling yet: run ipm_step, lp_solve or direction_solve first");
            return LP_EINVAL;
        }
        if (cls == LP_K_GRAM && !p->gsor) {
            set_error("no dense Gram path for this problem");
            return LP_EINVAL;
        }
        if (gs && p->opt.krylov != LP_ABGMRES && p->opt.krylov != LP_BAGMRES) {
            set_error("CGNE and MRNE keep no Krylov basis");
            return LP_EINVAL;
        }
        kg = std::min<int64_t>(kg, p->kmax - 1);
    }
    kg = std::max<int64_t>(kg, 0);
    if (B.dirty) {
        lp_status rc = B.refresh();
        if (rc != LP_OK) return rc;
    }
    for (int s = 0; s < B.cap; ++s) {
        KrylovCtl t{};
        t.done = 1;
        if (B.mem[s]) {
            t.done = 0;
            t.active = 1;
            t.kmax = 1;
            // the delayed form's update works on column k - 1 of the last finish
            t.k = gs ? (int32_t)kg + (cls == LP_K_GS_UPDATE && !B.L.ba ? 1 : 0) : 0;
            t.inv_h = 1.0;
            t.dg_nu = 1.0;
            t.omega_c = B.mem[s]->omega_c;
        }
        B.h_slot[s].ctl = t;
    }
    if (cls == LP_K_SPMV_CSR && B.L.inner != 3 && B.L.all_fuse) {
        // every instance's sweep forms u itself: this class has no launch
        *us_per_launch = 0.0;
        if (bytes_per_launch) *bytes_per_launch = 0.0;
        if (flops_per_launch) *flops_per_launch = 0.0;
        if (launches_per_group) *launches_per_group = 0;
        return LP_OK;
    }
    hipStream_t st = B.st;
    LPK_HIP(hipMemcpyAsync(B.d_slot, B.h_slot, sizeof(Slot) * B.cap, hipMemcpyHostToDevice, st));
    LPK_HIP(hipStreamSynchronize(st));
    if (!B.cap_st) LPK_HIP(hipStreamCreateWithFlags(&B.cap_st, hipStreamNonBlocking));
    const uint32_t mask = B.prof_mask;
    B.prof_mask = 0;
    double bytes = 0.0, flops = 0.0;
    int64_t launches = 0;
    B.count_bytes = &bytes;
    B.count_flops = &flops;
    B.count_launch = &launches;
    B.count_cls = cls;
    B.L.st = B.cap_st;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(B.cap_st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        if (cls == LP_K_SWEEP) {
            // as the AB-GMRES iteration launches it (with the product where fused)
            enqueue_precond(B, -1, false, 0, (B.L.krylov == LP_ABGMRES && !B.L.ba) ? 1 : 0);
        } else if (gs) {
            if (B.L.ba) enqueue_gs(B, kg, cls == LP_K_GS_DOTS ? GS_DOTS : GS_UPDATES);
            else enqueue_dgs(B, kg, cls == LP_K_GS_DOTS ? GS_DOTS : GS_UPDATES);
        } else if (cls == LP_K_SPMV_CSC) {
            if (B.L.inner != 3) {
                Prof pr(&B, LP_K_SPMV_CSC, -1, over_members(B, csc_bytes));
                b_spmv(B.L, M_AH_CSC, V_PCOL, V_Z64, EPI_PLAIN, -1, -1, 0, false);
            }
        } else if (cls == LP_K_SPMV_CSR) {
            if (B.L.inner == 3) {
                enqueue_products(B, -1);   // the dense path's only product, u = G p_k
            } else if (!B.L.all_fuse) {
                // the instances whose sweep does not form u itself
                Prof pr(&B, LP_K_SPMV_CSR, -1,
                        over_members(B, [](const lp_problem* p) { return fuses_u(p) ? 0.0 : csr_bytes(p); }));
                b_spmv(B.L, M_AH_CSR, V_Z64, V_U, EPI_PLAIN, -1, -1, B.L.any_fuse ? PM_NOFUSE : 0, false);
            }
        } else {
            for (int s = 0; s < B.cap; ++s)
                if (B.mem[s]) (void)build_dense_preconditioner(B, B.mem[s]);
        }
        e = hipStreamEndCapture(B.cap_st, &g);
    }
    B.L.st = st;
    B.prof_mask = mask;
    B.count_bytes = nullptr;
    B.count_flops = nullptr;
    B.count_launch = nullptr;
    B.count_cls = -1;
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

extern "C" lp_status lp_time_kernel(lp_problem* p, int32_t cls, int32_t reps, double* us_per_launch,
                                    double* bytes_per_launch, double* flops_per_launch,
                                    int32_t* launches_per_group) {
    if (!p) return LP_EINVAL;
    Batch* b = nullptr;
    lp_status rc = solo_batch(p, &b);
    if (rc != LP_OK) return rc;
    return time_kernel(*b, cls, reps, us_per_launch, bytes_per_launch, flops_per_launch, launches_per_group);
}

extern "C" lp_status lp_time_batch_kernel(lp_problem** problems, int32_t count, int32_t cls, int32_t reps,
                                          double* us_per_launch, double* bytes_per_launch,
                                          double* flops_per_launch, int32_t* launches_per_group) {
    if (!problems || count < 1) {
        set_error("NULL problems or count < 1");
        return LP_EINVAL;
    }
    for (int32_t i = 0; i < count; ++i) {
        if (!problems[i]) {
            set_error("NULL problem");
            return LP_EINVAL;
        }
        if (!batch_compatible(problems[0], problems[i])) {
            set_error("problems of one timed batch must share precision, inner iterations and layout");
            return LP_EINVAL;
        }
    }
    for (int32_t i = 0; i < count; ++i) LPK_HIP(hipStreamSynchronize(problems[i]->st));
    Batch B;
    lp_status rc = B.init(count, problems[0]->st, false);
    if (rc != LP_OK) return rc;
    for (int32_t i = 0; i < count; ++i) B.mem[i] = problems[i];
    rc = time_kernel(B, cls, reps, us_per_launch, bytes_per_launch, flops_per_launch, launches_per_group);
    (void)hipStreamSynchronize(B.st);
    return rc;
}
