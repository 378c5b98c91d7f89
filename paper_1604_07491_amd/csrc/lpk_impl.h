// Internal state of an lp_problem and of the batched engine.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/lpk.h"
#include "bounds.h"
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
// the sweeps of a problem with these options run in FP32 (LP_MIXED, where FP32 moves fewer
// bytes from memory or lets the sweep run from LDS alone): kind64 / kind32 are sweep_kind
// in FP64 / FP32
bool fp32_sweeps(const lp_options& o, bool gsor, int kind64, int kind32);
// host validation of lp_create's inputs (no device call)
lp_status validate_inputs(int64_t m, int64_t n, int64_t nnz, const int64_t* rp, const int32_t* ci,
                          const double* val, const double* b, const double* c);

// lanes per row for a row-dot over rows of mean length len
int lanes_for(double len);
// Gram-Schmidt rows per lane for m rows (chunks of 64 rpl rows, at most 1024 chunks)
int gs_rpl_for(int64_t m);
// Gram-Schmidt dot segments (1024 rows each) of an m-row basis
int gs_segments(int64_t m);
// the fused Gram-Schmidt updates need few dot segments and the coefficients in LDS
bool gs_fusable(int64_t m, int64_t kmax);

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
    int il;             // 0: a row's lanes are consecutive; else il rows per wave, interleaved
    int R;              // row elements per lane held in registers (8, 16 or 32)
    int maxlen;         // longest row
    int64_t nnz;        // nonzeros of the colour
    int slice0 = -1;    // sliced: first slice (else -1)
    int nslice = 0;     // sliced: slices of the colour
    int sR = 8;         // sliced: slot steps per lane held in registers (8, 12, 16 or 32)
};

// the lane layout of a colour's rows whose wave-wide loads touch fewer cache lines
void choose_layout(Colour& C, const int32_t* rp, const int32_t* ci, int zbytes);

// How the NE-SOR / NE-SSOR sweeps of an LP with these colours run (Inst::lds) with values
// of tb bytes: 2, one block per LP with the row data, z, v_k and p_k in LDS; 1, one block
// with z, v_k and p_k in LDS and the rows read from memory, when every colour's rows take
// at most LDS_ROUNDS_MAX rounds of the block's threads at no more than 8 elements a lane;
// 0, colour by colour over many blocks.
int sweep_kind(int64_t m, int64_t n, int64_t nnz, const std::vector<Colour>& cols, int tb);

// one timed launch: events a (before) and b (after) on the batch's stream
struct ProfRec {
    int cls;
    int64_t solve;      // which Krylov solve it belongs to
    int64_t iter;       // host-side iteration index inside that solve (-1: not a loop kernel)
    double bytes;
    double flops;
    hipEvent_t a, b;
};

// the per-instance control words the host reads back, and the phase parameters it writes
struct Slot {
    KrylovCtl ctl;
    double out[RED_NQ];
};
struct Param {
    double scal[SC_COUNT];
    int32_t mode;
    int32_t pad[3];
};

struct Batch;

}  // namespace lpk

struct lp_problem {
    int64_t m = 0, n = 0, nnz = 0;
    lp_options opt{};
    hipStream_t st = nullptr;
    int device = 0;
    bool dense = false;
    bool mixed = false;                             // FP32 sweeps (LP_MIXED where they pay)
    int lds_kind = 0;                               // sweep_kind of the NE-SOR / NE-SSOR sweeps
    bool gsor = false;                              // dense: SOR on the Gram matrix
    double* G = nullptr;                            // m x m Gram matrix A_hat A_hat^T
    double* Wgram = nullptr;                        // split-K partial tiles of the Gram build
    double *Xinv = nullptr, *Tmat = nullptr, *Tmat2 = nullptr, *Cmat = nullptr, *Rblk = nullptr;
    const double* Capply = nullptr;                 // the preconditioner matrix C<l>
    float* C32 = nullptr;

    // host-side structure
    std::vector<int32_t> perm;        // permuted row t is original row perm[t]
    std::vector<lpk::Colour> colours;
    std::vector<int32_t> h_cstart, h_cg, h_ctab;
    int g_csr = 64, g_csc = 1;
    int rpl = 1, nchunks = 1;
    bool zcover = false;                            // colour 0 covers every column

    lpk::DevArena arena;
    // structure and data (permuted rows)
    int32_t *rp = nullptr, *ci = nullptr, *cp = nullptr, *ri = nullptr, *perm_d = nullptr;
    int32_t *cstart = nullptr, *cg = nullptr;
    int32_t* ctab = nullptr;                        // one-block sweep colour table (lds_kind != 0)
    int32_t *cslice = nullptr, *soff = nullptr, *slen = nullptr, *rsl = nullptr, *sl_idx = nullptr, *srows = nullptr;
    int32_t nsl = 0;                                // slices over all colours
    int32_t* crow = nullptr;                        // rows not in slices
    int32_t ncrow = 0;
    double* sl_val = nullptr;                       // sliced copies of A_hat (see Inst)
    float* sl_val32 = nullptr;
    double *a = nullptr, *ac = nullptr;            // A values, CSR and CSC
    double *ah = nullptr, *ahc = nullptr;          // A_hat values, CSR and CSC
    float *ah32 = nullptr, *ahc32 = nullptr;       // FP32 copies (mixed precision)
    double* vec[lpk::V_COUNT] = {nullptr};         // vectors by selector
    float *z32 = nullptr, *r32 = nullptr;
    // Krylov workspace
    int64_t kmax = 0, ldv = 0, ldh = 0;
    double *V = nullptr, *P = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *gam = nullptr;
    double *ykr = nullptr, *h2 = nullptr;
    double* gpart = nullptr;                        // CGS pass-0 dot partials (segments x (kmax+1)), norm partials
    double* gpart2 = nullptr;                       // CGS pass-1 dot partials
    double norm_b = 0.0, norm_c = 0.0;
    // interior-point state
    bool have_point = false;
    lp_ipm_state ist{};
    std::vector<lp_iter_info> log;
    int64_t krylov_total = 0;
    double omega_c = 0.0;                           // Cimmino step of the current scaling
    // the batch of one that serves the single-problem entry points
    std::unique_ptr<lpk::Batch> solo;
    // lp_create_bounded: how the caller's variables sit in this standard form
    std::unique_ptr<lpk::BoundMap> bounds;
    int32_t* fpairs = nullptr;                      // device (x+ column, x- column) per free variable
    int32_t nfpairs = 0;
    ~lp_problem();
};

namespace lpk {

// A batch: up to `cap` problems whose phases run in lockstep, one launch per phase for all
// of them.  Descriptors live in device memory; the graph of Krylov iterations is captured
// for the current membership and replayed.
struct Batch {
    int cap = 0;
    hipStream_t st = nullptr;
    bool own_stream = false;
    int device = 0;
    std::vector<lp_problem*> mem;     // per slot; nullptr when empty
    Inst* d_inst = nullptr;
    std::vector<Inst> h_inst;
    Slot* d_slot = nullptr;
    Slot* h_slot = nullptr;           // pinned
    Param* d_param = nullptr;
    Param* h_param = nullptr;         // pinned
    double* d_part = nullptr;         // cap x RED_NQ x RED_MAXBLK
    BLaunch L{};
    std::vector<int> grid_colour;
    std::vector<char> colour_r;       // registers per lane of each colour launch (max over members)
    BLaunch graph_L{};                // the launch shapes the graph was captured with
    std::vector<int> graph_colour;
    std::vector<char> graph_r;
    bool dirty = true;                // membership changed since the descriptors were uploaded
    bool param_inflight = false;      // a parameter upload may still be in flight
    // captured Krylov iterations
    hipStream_t cap_st = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_iters = 0;
    // narrower captures of the same iterations for when few members iterate: width
    // cap >> (i + 1) for capture i, over d_inst_c (the iterating members' descriptors
    // first, then descriptors whose control block reads done)
    static constexpr int NARROW = 3;
    hipGraph_t graph_c[NARROW] = {};
    hipGraphExec_t gexec_c[NARROW] = {};
    Inst* d_inst_c = nullptr;
    Inst* h_inst_c = nullptr;         // pinned
    Slot* d_pad_slot = nullptr;       // what an empty slot holds, for the padding entries:
    Param* d_pad_param = nullptr;     // control block with done = 1, parameters, partials
    double* d_pad_part = nullptr;
    std::vector<int> c_slots;         // the members d_inst_c holds, in order (empty: none)
    int c_width = 0;
    int64_t last_iters = 0;           // polling hint
    // profiler (events on st) and launch accounting for timing captures
    uint32_t prof_mask = 0;
    double* count_bytes = nullptr;
    double* count_flops = nullptr;
    int64_t* count_launch = nullptr;
    int count_cls = -1;
    int64_t solve_id = 0;             // solves started on this batch
    int64_t cur_solve = -1;           // the solve the launches being enqueued belong to
    std::vector<ProfRec> prof_recs;
    std::vector<hipEvent_t> prof_pool;
    std::vector<int64_t> solve_iters;
    int64_t prof_launch[LP_K_COUNT] = {0};
    double prof_ms[LP_K_COUNT] = {0}, prof_bytes[LP_K_COUNT] = {0}, prof_flops[LP_K_COUNT] = {0};

    // device arrays (d_inst, d_inst_c, d_pad_*, d_slot, d_param, d_part) and host mirrors
    // (h_slot, h_param, h_inst_c) lent by the caller (init_external): never freed here
    bool external = false;

    ~Batch();
    lp_status init(int capacity, hipStream_t stream, bool own);
    // a batch of one on device memory at dev (BATCH_EXTERNAL_BYTES, 256-byte aligned) and
    // the given host mirrors; allocates nothing, and captures no graph
    lp_status init_external(hipStream_t stream, unsigned char* dev, Slot* hs, Param* hp, Inst* hic);
    int free_slot() const;
    int members() const;
    // make the device descriptors, launch maxima and graph match the membership
    lp_status refresh();
    void drop_graph();
    // upload the phase parameters of every slot (scal, mode)
    lp_status put_params();
    // read the control words and reduction results of every slot (synchronises the stream)
    lp_status get_slots();
};

// device bytes a batch of one takes in init_external: two descriptors, the padding slot,
// parameters and partials, the slot, parameters and partials, each 256-byte aligned
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t BATCH_EXTERNAL_BYTES = 2 * align256(sizeof(Inst)) + 2 * align256(sizeof(Slot)) +
                                        2 * align256(sizeof(Param)) +
                                        2 * align256(sizeof(double) * RED_NQ * RED_MAXBLK);

// homogeneity key: problems of one batch share these
bool batch_compatible(const lp_problem* a, const lp_problem* b);

// the batched Krylov solve (AB-GMRES with inner-iteration preconditioning, Sec. 3.2) for
// every slot whose mode has a bit of pmask: f = vec[V_F] (permuted rows) -> dw (V_DW) and
// the multipliers dyh (V_DYH, dw = A_hat^T dyh).  Tolerances from scal[SC_TOL].
lp_status krylov_batch(Batch& B, int pmask, std::vector<lp_krylov_info>* info);
// rho and A_hat for every slot with a bit of pmask (d = vec[V_D]); dense: G and C<l>;
// Cimmino: the step from the power iteration for slots marked MD_POW
lp_status scale_batch(Batch& B, int pmask);
lp_status build_dense_preconditioner(Batch& B, lp_problem* p);

// Interior-point driver over a batch.  Every member runs its own state machine (its own
// phase of Mehrotra's iteration or of the starting point); a round launches each phase's
// kernels once for all members in that phase, then Krylov iterations for every member
// inside a solve, then reads every member's scalars in one copy.  Members join and leave
// at any round.
struct Engine {
    enum State {
        EMPTY = 0, DONE,
        MEAS,       // residuals, error measure, stopping test
        SCALE,      // D, A_hat, first right-hand side; starts solve 1
        KRY1,       // inside solve 1
        FIN1,       // solve 1 assembled; direction recovery and ratio tests
        MUAF,       // mu_af at the predictor's step
        RHS2,       // second right-hand side; starts solve 2
        KRY2,       // inside solve 2
        FIN2,       // solve 2 assembled; corrector recovery / starting point y, s
        BT,         // back-tracking test
        UPD,        // the step (with the next point's measures unless step-wise)
        SH1, SH2,   // starting point: shifts
        RHS3,       // a centrality corrector's right-hand side; starts its solve
        KRY3,       // inside a centrality corrector's solve
        FIN3,       // its solve assembled; corrector recovery and ratio tests
        ST_COUNT
    };
    struct Member {
        lp_problem* p = nullptr;
        State state = EMPTY;
        bool init = false;            // role: computing the starting point
        int32_t limit_k = 0;          // evaluate only once ist.k reaches it
        lp_status status = LP_OK;
        int32_t iters = 0;
        int32_t steps = 0;            // interior-point steps taken in this engine
        lp_iter_info L{};             // the current iteration's log entry
        lp_iter_info last{};          // the final measures
        bool cc = false;
        double ap = 0.0, ad = 0.0;
        int32_t mcc = 0;              // centrality correctors tried in this step
        bool mcc_add = false;         // the last one was accepted: add it in the next round
        int32_t bt = 0;
        double t_join = 0.0, t_done = 0.0;
        int64_t k0 = 0;               // krylov_total at join
        int64_t solve_id = -1, enq = 0;   // profiler bookkeeping of the current solve
        int64_t last_k = 0;           // iterations of the member's previous solve
    };
    Batch* B = nullptr;
    std::vector<Member> mem;
    lp_status error = LP_OK;          // a device error stops the whole batch
    bool stepwise = false;            // ipm_step: the update round does not evaluate the next point
    bool issued = false;              // a round's work is queued and complete() has not run
    bool hold = false;                // this round's phases wait for the others' solves

    void attach(Batch* b);
    // join a free slot: start with the starting point, or from the point it holds
    int join(lp_problem* p, bool from_point, int32_t limit_k);
    // one round: issue() queues every launch of the round and the copy of the control words
    // on the batch's stream without waiting; complete() waits for them and advances each
    // member's state machine.  round() is the two in a row.  Members join and leave only
    // between complete() and the next issue().
    lp_status round();
    lp_status issue();
    lp_status complete();
    bool ready() const;               // nothing issued, or the issued round has finished
    bool any_live() const;
    void leave(int slot);             // empty a slot
};

double now_seconds();
void fill_result(const Engine::Member& mb, lp_result* r);

// profiler: bracket a launch of class cls with events when cls is enabled
struct Prof {
    Batch* B;
    int idx = -1;
    Prof(Batch* b, int cls, int64_t iter, double bytes, double flops = 0.0);
    ~Prof();
};
lp_status prof_collect(Batch& B);
void prof_release(Batch& B);

// the solo batch of a problem (created on first use, on the problem's stream)
lp_status solo_batch(lp_problem* p, Batch** out);

}  // namespace lpk
