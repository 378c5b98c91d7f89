// C ABI of the library: validation, problem set-up, and the entry points declared in
// include/lpk.h.  Host inputs are validated before any HIP call.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <new>
#include <string>
#include <vector>

#include "lpk_impl.h"

namespace lpk {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

lp_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string("HIP error ") + hipGetErrorString(e) + " in " + what;
    return LP_EDEVICE;
}

static lp_status fail(lp_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

static bool is_gmres(const lp_options& o) { return o.krylov == LP_ABGMRES || o.krylov == LP_BAGMRES; }

// Krylov iteration limit: m (Sec. 4.2) unless the options cap it; AB-GMRES keeps a basis
// and multiplier vector per iteration (BA-GMRES a basis vector), so its limit is also at
// most what fits in a 16 GiB budget for them
static int64_t plan_kmax(int64_t m, const lp_options& o) {
    int64_t k = m;
    if (o.krylov_max_iter > 0) k = std::min<int64_t>(k, o.krylov_max_iter);
    if (!is_gmres(o)) return std::max<int64_t>(1, k);
    const int64_t budget = (int64_t)16 << 30;
    const int64_t per = o.krylov == LP_ABGMRES ? 16 : 8;
    const int64_t cap = std::max<int64_t>(8, budget / (per * (m + 1)));
    return std::max<int64_t>(1, std::min(k, cap));
}

// columns of V (and the order of H): the basis for AB-GMRES and BA-GMRES, one column for
// CGNE and MRNE (the preconditioner's input)
static int64_t basis_cols(int64_t kmax, const lp_options& o) { return is_gmres(o) ? kmax + 1 : 1; }
// columns of P, the multipliers: one per basis vector for AB-GMRES; BA-GMRES keeps its
// multipliers in V_U and CGNE / MRNE in one column
static int64_t mult_cols(int64_t kmax, const lp_options& o) { return o.krylov == LP_ABGMRES ? kmax + 1 : 1; }

struct Sizes {
    uint64_t bytes = 0;
    void add(int64_t count, int64_t elem) {
        if (count <= 0) count = 1;
        bytes += ((uint64_t)count * (uint64_t)elem + 255) & ~(uint64_t)255;
    }
};

bool fp32_sweeps(const lp_options& o, bool gsor, int kind64, int kind32) {
    if (o.precision != LP_MIXED) return false;
    // FP32 pays where the FP64 NE-SOR / NE-SSOR sweep cannot run in one block from LDS: it
    // then halves the bytes of z and of the row values that stream from memory, and may
    // bring z (and the rows) into LDS.  FP64 sweeps leave z_k = A_hat^T p_k for free,
    // where FP32 sweeps need a product in FP64; for a sweep already in LDS, whose colour
    // steps are bound by latency, that product costs more than FP32 saves (measured on
    // the serving mix: staging in FP32 only, 3 % slower).  Cimmino and the dense path: FP32.
    (void)kind32;
    const bool sor = o.inner == LP_NESOR || o.inner == LP_NESSOR;
    if (gsor || !sor) return true;
    return kind64 == 0;
}

int sweep_kind(int64_t m, int64_t n, int64_t nnz, const std::vector<Colour>& cols, int tb) {
    const int64_t nc = (int64_t)cols.size();
    if (nc == 0) return 0;
    if (lds_stage_bytes(m, n, nnz, tb) <= LDS_STAGE_MAX) return 2;
    if (lds_z_bytes(m, n, tb) > LDS_Z_MAX) return 0;
    for (const Colour& C : cols) {
        const int64_t rounds = ((int64_t)(C.r1 - C.r0) * C.g + LDS_SWEEP_THREADS - 1) / LDS_SWEEP_THREADS;
        if (rounds > LDS_ROUNDS_MAX || C.maxlen > 8 * C.g) return 0;
    }
    return 1;
}

uint64_t footprint(int64_t m, int64_t n, int64_t nnz, const lp_options& o) {
    Sizes z;
    // An upper bound.  NE-SOR / NE-SSOR sweeps staged in LDS in FP64 (the staged size with
    // as many colours as rows still fits) run in FP64 from LDS: no FP32 copies, no row
    // slices.  Otherwise LP_MIXED may keep FP32 copies and the sweeps may need slices.
    const bool sor = o.inner == LP_NESOR || o.inner == LP_NESSOR;
    const bool staged64 = sor && lds_stage_bytes(m, n, nnz, 8) <= LDS_STAGE_MAX;
    const bool mixed = o.precision == LP_MIXED && !staged64;
    const int64_t kmax = plan_kmax(m, o);
    const int64_t cols = basis_cols(kmax, o), pcols = mult_cols(kmax, o);
    const bool cg = !is_gmres(o);
    const int64_t nchunks = (m + 64 * gs_rpl_for(m) - 1) / (64 * gs_rpl_for(m));
    z.add(m + 1, 4); z.add(nnz, 4); z.add(nnz, 8); z.add(n + 1, 4); z.add(nnz, 4); z.add(nnz, 8);
    z.add(nnz, 8); z.add(nnz, 8);
    if (mixed) { z.add(nnz, 4); z.add(nnz, 4); }
    z.add(m, 4);                                  // permutation
    z.add(m + 1, 4); z.add(m, 4);                 // colour ranges and lanes (at most m colours)
    z.add(4 * m, 4);                              // the one-block sweep's colour table
    if (sor && !staged64) {
        // row slices: at most 5/4 of the nonzeros with columns and values (FP32 copy in
        // mixed precision); slice starts of the colours, slice offsets and lengths, row
        // positions, slice rows, the other rows
        const int64_t np = nnz + nnz / 4 + 1;
        z.add(np, 4); z.add(np, 8);
        if (mixed) z.add(np, 4);
        z.add(m, 4); z.add(m, 4); z.add(m, 4); z.add(m, 4); z.add(2 * m, 4); z.add(m, 4);
    }
    for (int i = 0; i < (cg ? 15 : 12); ++i) z.add(m, 8);    // m-vectors
    for (int i = 0; i < (cg ? 14 : 11); ++i) z.add(n, 8);    // n-vectors
    if (o.max_correctors > 0) { z.add(n, 8); z.add(n, 8); }  // a corrector's dx, ds
    z.add(n, 4); z.add(m, 4);                     // z32, r32
    z.add(m * cols, 8); z.add(m * pcols, 8);      // V, P
    z.add(cols * cols, 8);                        // H
    for (int i = 0; i < 5; ++i) z.add(cols + 1, 8);
    if (cg) {
        z.add(nchunks, 8);
    } else {
        z.add(std::max<int64_t>(nchunks, (int64_t)gs_segments(m) * (cols + 1)), 8);
        z.add((int64_t)gs_segments(m) * (cols + 1), 8);
    }
    // the problem's batch of one: descriptor, control words, parameters, partials
    z.add(1, sizeof(Inst)); z.add(1, sizeof(Slot)); z.add(1, sizeof(Param));
    z.add((int64_t)RED_NQ * RED_MAXBLK, 8);
    return z.bytes;
}

// Distinct 128-byte lines touched by the wave-wide loads of z, values and indices, summed
// over the element steps of the first waves of a colour, per element.  il = 0: a row's g
// lanes are consecutive; il > 0: il rows per wave, lane l on row l mod il.
static double line_cost(const Colour& C, const int32_t* rp, const int32_t* ci, int g, int il, int zbytes) {
    const int rows_per_wave = il ? il : 64 / g;
    const int gl = il ? 64 / il : g;
    double lines = 0.0, elems = 0.0;
    std::vector<int64_t> zl, vl, xl;
    for (int w = 0; w < 8; ++w) {
        const int64_t base = (int64_t)C.r0 + (int64_t)w * rows_per_wave;
        if (base >= C.r1) break;
        for (int t = 0;; ++t) {
            zl.clear();
            vl.clear();
            xl.clear();
            for (int l = 0; l < 64; ++l) {
                const int64_t row = il ? base + (l % il) : base + l / g;
                const int slot = il ? l / il : l % g;
                if (row >= C.r1) continue;
                const int64_t kk = rp[row] + slot + (int64_t)t * gl;
                if (kk >= rp[row + 1]) continue;
                zl.push_back((int64_t)ci[kk] * zbytes / 128);
                vl.push_back(kk * zbytes / 128);
                xl.push_back(kk * 4 / 128);
                elems += 1.0;
            }
            if (zl.empty()) break;
            for (std::vector<int64_t>* v : {&zl, &vl, &xl}) {
                std::sort(v->begin(), v->end());
                lines += (double)(std::unique(v->begin(), v->end()) - v->begin());
            }
        }
    }
    return elems > 0.0 ? lines / elems : 0.0;
}

// Slices of SL_ROWS rows for colour C, stored slot-major from offset off0 (see Inst): built
// (true) when the wave-wide loads of the sliced kernel touch under 0.6 of the lines per
// element that the colour's CSR lane layout touches, padding adds at most a quarter to the
// colour's elements and every offset stays below 2^31.
static bool slice_colour(Colour& C, const int32_t* rp, const int32_t* ci, int zbytes, std::vector<int32_t>& soff,
                         std::vector<int32_t>& slen, std::vector<int32_t>& srows, std::vector<int32_t>& rsl,
                         std::vector<int32_t>& sidx) {
    const int64_t rows = C.r1 - C.r0;
    const int64_t nsl = (rows + SL_ROWS - 1) / SL_ROWS;
    std::vector<int32_t> ls((size_t)nsl);
    int64_t padded = 0;
    for (int64_t q = 0; q < nsl; ++q) {
        int len = 0;
        for (int64_t t = C.r0 + q * SL_ROWS; t < std::min<int64_t>(C.r1, C.r0 + (q + 1) * SL_ROWS); ++t)
            len = std::max<int>(len, rp[t + 1] - rp[t]);
        ls[q] = (len + SL_GROUPS - 1) / SL_GROUPS * SL_GROUPS;
        padded += (int64_t)ls[q] * SL_ROWS;
    }
    const int64_t off0 = (int64_t)sidx.size();
    if (padded * 4 > C.nnz * 5 || off0 + padded >= ((int64_t)1 << 31)) return false;
    // lines per element over the first slices' loads
    double lines = 0.0, elems = 0.0;
    std::vector<int64_t> zl, vl, xl;
    int64_t off = off0;
    for (int64_t q = 0; q < std::min<int64_t>(nsl, 8); ++q) {
        for (int wv = 0; wv < SL_THREADS / 64; ++wv)
            for (int t = 0; t * SL_GROUPS < ls[q]; ++t) {
                zl.clear();
                vl.clear();
                xl.clear();
                for (int l = 0; l < 64; ++l) {
                    const int r = l % SL_ROWS, slot = wv * (64 / SL_ROWS) + l / SL_ROWS + t * SL_GROUPS;
                    const int64_t pos = off + (int64_t)slot * SL_ROWS + r;
                    vl.push_back(pos * zbytes / 128);
                    xl.push_back(pos * 4 / 128);
                    const int64_t row = C.r0 + q * SL_ROWS + r;
                    if (row < C.r1 && slot < rp[row + 1] - rp[row]) {
                        zl.push_back((int64_t)ci[rp[row] + slot] * zbytes / 128);
                        elems += 1.0;
                    }
                }
                for (std::vector<int64_t>* v : {&zl, &vl, &xl}) {
                    std::sort(v->begin(), v->end());
                    lines += (double)(std::unique(v->begin(), v->end()) - v->begin());
                }
            }
        off += (int64_t)ls[q] * SL_ROWS;
    }
    const double cur = line_cost(C, rp, ci, C.il ? 64 / C.il : C.g, C.il, zbytes);
    if (elems == 0.0 || lines / elems >= 0.6 * cur) return false;
    C.slice0 = (int)soff.size();
    C.nslice = (int)nsl;
    int steps = 0;
    sidx.resize((size_t)(off0 + padded), -1);
    off = off0;
    for (int64_t q = 0; q < nsl; ++q) {
        soff.push_back((int32_t)off);
        slen.push_back(ls[q]);
        srows.push_back((int32_t)(C.r0 + q * SL_ROWS));
        srows.push_back((int32_t)std::min<int64_t>(SL_ROWS, C.r1 - C.r0 - q * SL_ROWS));
        steps = std::max(steps, ls[q] / SL_GROUPS);
        for (int r = 0; r < SL_ROWS; ++r) {
            const int64_t row = C.r0 + q * SL_ROWS + r;
            if (row >= C.r1) break;
            rsl[row] = (int32_t)(off + r);
            for (int32_t k = rp[row]; k < rp[row + 1]; ++k) sidx[off + (int64_t)(k - rp[row]) * SL_ROWS + r] = ci[k];
        }
        off += (int64_t)ls[q] * SL_ROWS;
    }
    C.sR = steps <= 8 ? 8 : steps <= 12 ? 12 : steps <= 16 ? 16 : 32;
    return true;
}

// registers per lane for a row of len elements over g lanes: 8, 16 or 32 (longer rows
// are streamed twice)
static int regs_for(int len, int g) {
    const int need = (len + g - 1) / g;
    return need <= 8 ? 8 : need <= 16 ? 16 : 32;
}

// the fewest rows per wave (the most lanes per row, the shortest serial chain per lane)
// whose loads touch under 3/4 of the lines of the consecutive layout.  (Taking the layout
// with the fewest lines instead, 4 transportation sinks per wave with 32 registers per
// lane, measured 15 % slower than 2 sinks per wave with 16.)
void choose_layout(Colour& C, const int32_t* rp, const int32_t* ci, int zbytes) {
    C.il = 0;
    if (C.g < 16) return;
    const double cont = line_cost(C, rp, ci, C.g, 0, zbytes);
    for (int il = 2; il <= 8; il *= 2) {
        if (line_cost(C, rp, ci, 64 / il, il, zbytes) < 0.75 * cont) {
            C.il = il;
            C.g = 64 / il;
            break;
        }
    }
    C.R = regs_for(C.maxlen, C.g);
}

static lp_status validate(int64_t m, int64_t n, int64_t nnz, const int64_t* rp, const int32_t* ci,
                          const double* val, bool need_m_le_n = true) {
    if (m < 1 || n < 1) return fail(LP_EDIM, "m and n must be positive");
    if (need_m_le_n && m > n) return fail(LP_EDIM, "m > n: the problem statement assumes m <= n");
    if (nnz < 1 || nnz >= ((int64_t)1 << 31) || n >= ((int64_t)1 << 31))
        return fail(LP_EDIM, "nnz and n must be below 2^31");
    if (!rp || !ci || !val) return fail(LP_EINVAL, "NULL CSR array");
    if (rp[0] != 0 || rp[m] != nnz) return fail(LP_EINVAL, "row_ptr must start at 0 and end at nnz");
    std::vector<char> colseen((size_t)n, 0);
    for (int64_t i = 0; i < m; ++i) {
        if (rp[i + 1] < rp[i]) return fail(LP_EINVAL, "row_ptr is decreasing at row " + std::to_string(i));
        if (rp[i + 1] == rp[i]) return fail(LP_EINVAL, "row " + std::to_string(i) + " is empty");
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t j = ci[k];
            if (j < 0 || j >= n) return fail(LP_EINVAL, "column index out of range in row " + std::to_string(i));
            if (k > rp[i] && ci[k - 1] >= j)
                return fail(LP_EINVAL, "column indices not strictly increasing in row " + std::to_string(i));
            if (!std::isfinite(val[k])) return fail(LP_ENONFINITE, "non-finite entry in A");
            colseen[j] = 1;
        }
    }
    for (int64_t j = 0; j < n; ++j)
        if (!colseen[j]) return fail(LP_EINVAL, "column " + std::to_string(j) + " is empty");
    return LP_OK;
}

static lp_status check_vec(const double* v, int64_t len, const char* name) {
    if (!v) return fail(LP_EINVAL, std::string("NULL ") + name);
    for (int64_t i = 0; i < len; ++i)
        if (!std::isfinite(v[i])) return fail(LP_ENONFINITE, std::string("non-finite entry in ") + name);
    return LP_OK;
}

lp_status validate_inputs(int64_t m, int64_t n, int64_t nnz, const int64_t* rp, const int32_t* ci,
                          const double* val, const double* b, const double* c) {
    lp_status rc = validate(m, n, nnz, rp, ci, val);
    if (rc != LP_OK) return rc;
    if ((rc = check_vec(b, m, "b")) != LP_OK) return rc;
    return check_vec(c, n, "c");
}

static lp_status check_device() {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) return fail(LP_EDEVICE, "no HIP device available");
    return LP_OK;
}

// copy a caller array (host or device per device_io) into a host vector
template <typename T>
static lp_status fetch(const T* src, int64_t count, bool dev, std::vector<T>& out) {
    out.resize((size_t)std::max<int64_t>(count, 0));
    if (count <= 0) return LP_OK;
    if (dev) LPK_HIP(hipMemcpy(out.data(), src, sizeof(T) * count, hipMemcpyDeviceToHost));
    else memcpy(out.data(), src, sizeof(T) * count);
    return LP_OK;
}

static void destroy(lp_problem* p) {
    if (!p) return;
    if (p->st) (void)hipStreamSynchronize(p->st);
    delete p;
}

// set-up from host arrays that have passed validation
static lp_status setup(lp_problem* p, const int64_t* rp, const int32_t* ci, const double* val,
                       const double* b, const double* c) {
    const int64_t m = p->m, n = p->n, nnz = p->nnz;
    // colouring and the permuted CSR (a dense A is a complete conflict graph: colour =
    // row, the natural order)
    std::vector<int32_t> colour((size_t)m);
    p->perm.resize((size_t)m);
    int32_t ncol;
    if (p->dense) {
        for (int64_t i = 0; i < m; ++i) colour[i] = p->perm[i] = (int32_t)i;
        ncol = (int32_t)m;
    } else {
        ncol = greedy_colour(m, n, rp, ci, colour.data(), p->perm.data());
    }
    std::vector<int32_t> prp((size_t)m + 1), pci((size_t)nnz);
    std::vector<double> pa((size_t)nnz), pb((size_t)m);
    prp[0] = 0;
    for (int64_t t = 0; t < m; ++t) {
        const int64_t i = p->perm[t];
        const int64_t len = rp[i + 1] - rp[i];
        memcpy(&pci[prp[t]], ci + rp[i], sizeof(int32_t) * len);
        memcpy(&pa[prp[t]], val + rp[i], sizeof(double) * len);
        prp[t + 1] = (int32_t)(prp[t] + len);
        pb[t] = b[i];
    }
    // colour ranges and lanes per row for each colour
    p->colours.clear();
    int64_t t0 = 0;
    for (int32_t cl = 0; cl < ncol; ++cl) {
        int64_t t1 = t0;
        while (t1 < m && colour[p->perm[t1]] == cl) ++t1;
        Colour C;
        C.r0 = (int32_t)t0;
        C.r1 = (int32_t)t1;
        C.g = lanes_for((double)(prp[t1] - prp[t0]) / (double)std::max<int64_t>(1, t1 - t0));
        C.il = 0;
        C.nnz = prp[t1] - prp[t0];
        C.maxlen = 0;
        for (int64_t t = t0; t < t1; ++t) C.maxlen = std::max<int>(C.maxlen, prp[t + 1] - prp[t]);
        C.R = regs_for(C.maxlen, C.g);
        p->colours.push_back(C);
        t0 = t1;
    }
    // the sweep precision and where the sweeps run
    const bool sor = p->opt.inner == LP_NESOR || p->opt.inner == LP_NESSOR;
    const int kind64 = sweep_kind(m, n, nnz, p->colours, 8), kind32 = sweep_kind(m, n, nnz, p->colours, 4);
    const bool mixed = p->mixed = fp32_sweeps(p->opt, p->gsor, kind64, kind32);
    p->lds_kind = (sor && !p->gsor && !p->dense) ? (mixed ? kind32 : kind64) : 0;
    // one-block sweeps: at most LDS_LANES_MAX lanes a row when the longest row then needs at
    // most LDS_SLOTS slots a lane (fewer waves per colour, and a row's sum stays in DPP moves)
    if (p->lds_kind != 0)
        for (Colour& C : p->colours)
            if (C.g > LDS_LANES_MAX && (C.maxlen + LDS_LANES_MAX - 1) / LDS_LANES_MAX <= LDS_SLOTS) C.g = LDS_LANES_MAX;
    // lane layout by cache-line count, for LPs swept colour by colour (z in HBM)
    if (p->lds_kind == 0)
        for (Colour& C : p->colours) choose_layout(C, prp.data(), pci.data(), mixed ? 4 : 8);
    // slices for the colours whose neighbouring rows touch neighbouring columns (NE-SOR /
    // NE-SSOR swept colour by colour)
    std::vector<int32_t> h_cslice, h_soff, h_slen, h_srows, h_rsl, h_sidx, h_crow;
    {
        if (sor && !p->gsor && p->lds_kind == 0) {
            h_cslice.assign(p->colours.size(), -1);
            h_rsl.assign((size_t)m, -1);
            bool any = false;
            for (size_t cl = 0; cl < p->colours.size(); ++cl) {
                Colour& C = p->colours[cl];
                if (C.g >= 16 && slice_colour(C, prp.data(), pci.data(), mixed ? 4 : 8, h_soff, h_slen, h_srows, h_rsl, h_sidx)) {
                    h_cslice[cl] = C.slice0;
                    any = true;
                }
            }
            if (!any) h_cslice.clear();
        }
    }
    // does colour 0 touch every column? (then its first sweep sets z without clearing it)
    {
        std::vector<char> hit((size_t)n, 0);
        int64_t cnt = 0;
        if (!p->colours.empty())
            for (int64_t k = prp[p->colours[0].r0]; k < prp[p->colours[0].r1]; ++k)
                if (!hit[pci[k]]) {
                    hit[pci[k]] = 1;
                    ++cnt;
                }
        p->zcover = cnt == n;
    }
    // CSC of the permuted matrix (row indices in the permuted numbering, ascending)
    std::vector<int32_t> pcp((size_t)n + 1, 0), pri((size_t)nnz);
    std::vector<double> pac((size_t)nnz);
    for (int64_t k = 0; k < nnz; ++k) pcp[pci[k] + 1]++;
    for (int64_t j = 0; j < n; ++j) pcp[j + 1] += pcp[j];
    {
        std::vector<int32_t> fillp(pcp.begin(), pcp.end() - 1);
        for (int64_t t = 0; t < m; ++t)
            for (int32_t k = prp[t]; k < prp[t + 1]; ++k) {
                const int32_t pos = fillp[pci[k]]++;
                pri[pos] = (int32_t)t;
                pac[pos] = pa[k];
            }
    }
    p->g_csr = lanes_for((double)nnz / (double)m);
    p->g_csc = lanes_for((double)nnz / (double)n);
    double nb = 0.0, nc = 0.0;
    for (int64_t i = 0; i < m; ++i) nb += b[i] * b[i];
    for (int64_t j = 0; j < n; ++j) nc += c[j] * c[j];
    p->norm_b = std::sqrt(nb);
    p->norm_c = std::sqrt(nc);

    // device memory
    DevArena& A = p->arena;
    p->kmax = plan_kmax(m, p->opt);
    const int64_t cols = basis_cols(p->kmax, p->opt), pcols = mult_cols(p->kmax, p->opt);
    const bool cg = !is_gmres(p->opt);
    p->ldv = m;
    p->ldh = cols;
    p->rpl = gs_rpl_for(m);
    p->nchunks = (int)((m + 64 * p->rpl - 1) / (64 * p->rpl));
    p->rp = A.alloc<int32_t>(m + 1);
    p->ci = A.alloc<int32_t>(nnz);
    p->a = A.alloc<double>(nnz);
    p->cp = A.alloc<int32_t>(n + 1);
    p->ri = A.alloc<int32_t>(nnz);
    p->ac = A.alloc<double>(nnz);
    p->ah = A.alloc<double>(nnz);
    p->ahc = A.alloc<double>(nnz);
    if (mixed) {
        p->ah32 = A.alloc<float>(nnz);
        p->ahc32 = A.alloc<float>(nnz);
    }
    p->perm_d = A.alloc<int32_t>(m);
    p->cstart = A.alloc<int32_t>((int64_t)p->colours.size() + 1);
    p->cg = A.alloc<int32_t>((int64_t)p->colours.size());
    if (p->lds_kind != 0) p->ctab = A.alloc<int32_t>(4 * (int64_t)p->colours.size());
    if (!h_cslice.empty()) {
        p->cslice = A.alloc<int32_t>((int64_t)h_cslice.size());
        p->soff = A.alloc<int32_t>((int64_t)h_soff.size());
        p->slen = A.alloc<int32_t>((int64_t)h_slen.size());
        p->srows = A.alloc<int32_t>((int64_t)h_srows.size());
        p->nsl = (int32_t)h_soff.size();
        for (int64_t t = 0; t < m; ++t)
            if (h_rsl[t] < 0) h_crow.push_back((int32_t)t);
        p->ncrow = (int32_t)h_crow.size();
        p->crow = A.alloc<int32_t>(std::max<int64_t>(1, p->ncrow));
        p->rsl = A.alloc<int32_t>(m);
        p->sl_idx = A.alloc<int32_t>((int64_t)h_sidx.size());
        p->sl_val = A.alloc<double>((int64_t)h_sidx.size());
        if (mixed) p->sl_val32 = A.alloc<float>((int64_t)h_sidx.size());
    }
    const int mv[] = {V_Y, V_RHO, V_RP, V_DYA, V_DYC, V_F, V_DYH, V_TMPM, V_B, V_FH, V_U, V_R64};
    for (int q : mv) p->vec[q] = A.alloc<double>(m);
    const int nv[] = {V_X, V_S, V_D, V_RD, V_TN, V_DXA, V_DSA, V_DW, V_TMPN, V_C, V_Z64};
    for (int q : nv) p->vec[q] = A.alloc<double>(n);
    if (cg) {
        for (int q : {V_DYB, V_QM, V_PM}) p->vec[q] = A.alloc<double>(m);
        for (int q : {V_Q, V_PV, V_DWB}) p->vec[q] = A.alloc<double>(n);
    }
    if (p->opt.max_correctors > 0)
        for (int q : {V_DXC, V_DSC}) p->vec[q] = A.alloc<double>(n);
    p->z32 = A.alloc<float>(n);
    p->r32 = A.alloc<float>(m);
    p->V = A.alloc<double>(m * cols);
    p->P = A.alloc<double>(m * pcols);
    p->H = A.alloc<double>(cols * cols);
    p->cs = A.alloc<double>(cols + 1);
    p->sn = A.alloc<double>(cols + 1);
    p->gam = A.alloc<double>(cols + 1);
    p->ykr = A.alloc<double>(cols + 1);
    p->h2 = A.alloc<double>(cols + 1);
    if (cg) {
        p->gpart = A.alloc<double>(p->nchunks);
    } else {
        // Gram-Schmidt dot partials: segments x (cols + 1) (the delayed form adds u . u)
        p->gpart = A.alloc<double>(std::max<int64_t>(p->nchunks, (int64_t)gs_segments(m) * (cols + 1)));
        p->gpart2 = A.alloc<double>((int64_t)gs_segments(m) * (cols + 1));
    }
    if (p->gsor) {
        p->G = A.alloc<double>(m * m);
        if (gram_work_doubles((int)m) > 0) p->Wgram = A.alloc<double>(gram_work_doubles((int)m));
        p->Xinv = A.alloc<double>(m * m);
        p->Rblk = A.alloc<double>(64 * m);
        if (p->opt.inner_sweeps > 1) {
            p->Tmat = A.alloc<double>(m * m);
            p->Cmat = A.alloc<double>(m * m);
            if (p->opt.inner_sweeps > 2) p->Tmat2 = A.alloc<double>(m * m);
        }
        if (mixed) p->C32 = A.alloc<float>(m * m);
    }
    if (A.failed) return fail(LP_ENOMEM, "device allocation failed");
    hipStream_t st = p->st;
    p->h_cstart.resize(p->colours.size() + 1);
    p->h_cg.resize(p->colours.size());
    for (size_t cl = 0; cl < p->colours.size(); ++cl) {
        p->h_cstart[cl] = p->colours[cl].r0;
        p->h_cg[cl] = p->colours[cl].il ? -p->colours[cl].g : p->colours[cl].g;
    }
    p->h_cstart[p->colours.size()] = (int32_t)m;
    if (p->ctab) {
        std::vector<int32_t>& h_ctab = p->h_ctab;
        h_ctab.assign(4 * p->colours.size(), 0);
        for (size_t cl = 0; cl < p->colours.size(); ++cl) {
            const Colour& C = p->colours[cl];
            const int slots = slot_class((C.maxlen + C.g - 1) / C.g);
            h_ctab[4 * cl] = C.r0;
            h_ctab[4 * cl + 1] = C.r1;
            h_ctab[4 * cl + 2] = C.g;
            h_ctab[4 * cl + 3] = ((int64_t)(C.r1 - C.r0) * C.g <= 64 ? 1 : 0) | (slots << 1);
        }
        LPK_HIP(hipMemcpyAsync(p->ctab, h_ctab.data(), sizeof(int32_t) * h_ctab.size(), hipMemcpyHostToDevice, st));
    }
    LPK_HIP(hipMemcpyAsync(p->cstart, p->h_cstart.data(), sizeof(int32_t) * p->h_cstart.size(), hipMemcpyHostToDevice, st));
    if (!p->h_cg.empty())
        LPK_HIP(hipMemcpyAsync(p->cg, p->h_cg.data(), sizeof(int32_t) * p->h_cg.size(), hipMemcpyHostToDevice, st));
    if (p->cslice) {
        LPK_HIP(hipMemcpyAsync(p->cslice, h_cslice.data(), sizeof(int32_t) * h_cslice.size(), hipMemcpyHostToDevice, st));
        LPK_HIP(hipMemcpyAsync(p->soff, h_soff.data(), sizeof(int32_t) * h_soff.size(), hipMemcpyHostToDevice, st));
        LPK_HIP(hipMemcpyAsync(p->slen, h_slen.data(), sizeof(int32_t) * h_slen.size(), hipMemcpyHostToDevice, st));
        LPK_HIP(hipMemcpyAsync(p->srows, h_srows.data(), sizeof(int32_t) * h_srows.size(), hipMemcpyHostToDevice, st));
        if (p->ncrow > 0)
            LPK_HIP(hipMemcpyAsync(p->crow, h_crow.data(), sizeof(int32_t) * h_crow.size(), hipMemcpyHostToDevice, st));
        LPK_HIP(hipMemcpyAsync(p->rsl, h_rsl.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
        LPK_HIP(hipMemcpyAsync(p->sl_idx, h_sidx.data(), sizeof(int32_t) * h_sidx.size(), hipMemcpyHostToDevice, st));
        // padding values stay 0 (the scaling writes only the real elements)
        LPK_HIP(hipMemsetAsync(p->sl_val, 0, sizeof(double) * h_sidx.size(), st));
        if (p->sl_val32) LPK_HIP(hipMemsetAsync(p->sl_val32, 0, sizeof(float) * h_sidx.size(), st));
    }
    LPK_HIP(hipMemcpyAsync(p->rp, prp.data(), sizeof(int32_t) * (m + 1), hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemcpyAsync(p->ci, pci.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemcpyAsync(p->a, pa.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemcpyAsync(p->cp, pcp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemcpyAsync(p->ri, pri.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemcpyAsync(p->ac, pac.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemcpyAsync(p->perm_d, p->perm.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemcpyAsync(p->vec[V_B], pb.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemcpyAsync(p->vec[V_C], c, sizeof(double) * n, hipMemcpyHostToDevice, st));
    LPK_HIP(hipMemsetAsync(p->H, 0, sizeof(double) * cols * cols, st));
    LPK_HIP(hipStreamSynchronize(st));
    p->ist.eps_in = p->opt.eps_in0;
    return LP_OK;
}

static lp_status check_options(const lp_options& o, bool dense) {
    if (o.precision != LP_FP64 && o.precision != LP_MIXED) return fail(LP_EINVAL, "unknown precision");
    if (o.krylov != LP_ABGMRES && o.krylov != LP_CGNE && o.krylov != LP_MRNE && o.krylov != LP_BAGMRES)
        return fail(LP_EINVAL, "unknown Krylov method");
    // BA-GMRES applies the sweeps to m-vectors in place (input V_U, multipliers V_U);
    // the Cimmino and dense kernels and the FP32 sweeps keep their AB-GMRES layout
    if (o.krylov == LP_BAGMRES && (dense || (o.inner != LP_NESOR && o.inner != LP_NESSOR)))
        return fail(LP_EINVAL, "BA-GMRES needs sparse NE-SOR or NE-SSOR inner iterations");
    if (o.krylov == LP_BAGMRES && o.precision != LP_FP64)
        return fail(LP_EINVAL, "BA-GMRES needs FP64 inner iterations (precision LP_FP64)");
    if (o.inner != LP_NESOR && o.inner != LP_NESSOR && o.inner != LP_CIMMINO && !(dense && o.inner == LP_GSOR))
        return fail(LP_EINVAL, "inner iterations must be NE-SOR, NE-SSOR or Cimmino (or G-SOR for a dense A)");
    if (!is_gmres(o) && dense && (o.inner == LP_NESOR || o.inner == LP_GSOR))
        return fail(LP_EINVAL, "CGNE and MRNE need sparse sweeps: with a dense A use NE-SSOR or Cimmino");
    // MRNE forms q_k = A_hat^T C g_k by recurrence, which holds only while C is one fixed
    // linear map; FP32 sweeps perturb C at every application and the recurrence drifts
    // until the iteration diverges (CGNE recomputes its direction from C g_k each step)
    if (o.krylov == LP_MRNE && o.precision == LP_MIXED)
        return fail(LP_EINVAL, "MRNE needs FP64 inner iterations (precision LP_FP64)");
    if (o.inner_sweeps < 1 || o.inner_sweeps > 64) return fail(LP_EINVAL, "inner_sweeps must be in [1, 64]");
    if (o.max_correctors < 0 || o.max_correctors > 8) return fail(LP_EINVAL, "max_correctors must be in [0, 8]");
    if (!(o.omega > 0.0 && o.omega < 2.0)) return fail(LP_EINVAL, "omega must be in (0, 2)");
    if (!(o.eta >= 0.9 && o.eta < 1.0)) return fail(LP_EINVAL, "eta must be in [0.9, 1)");
    if (o.ipm_max_iter < 0) return fail(LP_EINVAL, "ipm_max_iter must be >= 0");
    if (o.schedule < 0 || o.schedule > 2) return fail(LP_EINVAL, "schedule must be 0, 1 or 2");
    if (!(o.eps_in_min > 0.0 && o.eps_in_min <= o.eps_in_max)) return fail(LP_EINVAL, "bad eps_in range");
    return LP_OK;
}

// the bounded-variable reduction of caller arrays already on the host: validation (the
// original problem may have m > n), then the standard form
static lp_status bounded_standard(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci,
                                  const double* val, const double* b, const double* c, const double* lo,
                                  const double* hi, StdForm& sf, BoundMap& bm) {
    if (!rp || !ci || !val || !lo || !hi) return fail(LP_EINVAL, "NULL input array");
    if (m < 1 || n < 1) return fail(LP_EDIM, "m and n must be positive");
    lp_status rc = validate(m, n, rp[m], rp, ci, val, false);
    if (rc != LP_OK) return rc;
    if ((rc = check_vec(b, m, "b")) != LP_OK) return rc;
    if ((rc = check_vec(c, n, "c")) != LP_OK) return rc;
    std::string err;
    if (!bounds_to_standard(m, n, rp, ci, val, b, c, lo, hi, sf, bm, err)) return fail(LP_EINVAL, err);
    if (sf.rp.back() >= ((int64_t)1 << 31) || sf.n >= ((int64_t)1 << 31))
        return fail(LP_EDIM, "the standard form has 2^31 or more nonzeros or columns");
    return LP_OK;
}

static lp_status copy_out(lp_problem* p, const double* dev, double* dst, int64_t len) {
    const hipMemcpyKind k = p->opt.device_io ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    LPK_HIP(hipMemcpyAsync(dst, dev, sizeof(double) * len, k, p->st));
    return LP_OK;
}

static lp_status copy_in(lp_problem* p, const double* src, double* dev, int64_t len) {
    const hipMemcpyKind k = p->opt.device_io ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    LPK_HIP(hipMemcpyAsync(dev, src, sizeof(double) * len, k, p->st));
    return LP_OK;
}

}  // namespace lpk

using namespace lpk;

extern "C" {

lp_status lp_options_default(lp_options* o) {
    if (!o) return fail(LP_EINVAL, "NULL options");
    memset(o, 0, sizeof(*o));
    o->precision = LP_FP64;
    o->krylov = LP_ABGMRES;
    o->inner = LP_NESOR;
    o->inner_sweeps = 2;
    o->omega = 1.0;
    o->omega_c = 0.0;
    o->krylov_max_iter = 0;
    o->ipm_max_iter = 99;
    o->start = 0;
    o->eps_out = 1e-8;
    o->eta = 0.9995;
    o->phi = 1e-5;
    o->sigma_max = 0.208;
    o->eps_in0 = 1e-6;
    o->eps_in_min = 1e-14;
    o->eps_in_max = 1e-4;
    o->init_tol = 1e-10;
    o->backtrack = 0.95;
    o->max_backtrack = 200;
    o->device_io = 0;
    o->stream = nullptr;
    o->poll_every = 0;
    o->use_graphs = 1;
    return LP_OK;
}

// host_inputs: the arrays are host arrays whatever opt.device_io says (the bounded-variable
// entry point passes its standard form); the problem keeps the caller's device_io
static lp_status create_impl(int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                             const int32_t* col_idx, const double* val, const double* b,
                             const double* c, const lp_options* o, bool dense, lp_problem** out,
                             bool host_inputs = false) {
    g_err.clear();
    if (!out) return fail(LP_EINVAL, "NULL out");
    *out = nullptr;
    lp_options opt;
    if (o) opt = *o;
    else lp_options_default(&opt);
    lp_status rc = check_options(opt, dense);
    if (rc != LP_OK) return rc;
    if (m < 1 || n < 1) return fail(LP_EDIM, "m and n must be positive");
    if (m > n) return fail(LP_EDIM, "m > n: the problem statement assumes m <= n");
    if (!row_ptr || !col_idx || !val || !b || !c) return fail(LP_EINVAL, "NULL input array");
    std::vector<int64_t> hrp;
    std::vector<int32_t> hci;
    std::vector<double> hval, hb, hc;
    const bool dev = opt.device_io != 0 && !host_inputs;
    if (dev) {
        rc = check_device();
        if (rc != LP_OK) return rc;
        if ((rc = fetch(row_ptr, m + 1, true, hrp)) != LP_OK) return rc;
        if (hrp[m] < 1 || hrp[m] >= ((int64_t)1 << 31)) return fail(LP_EDIM, "nnz must be in [1, 2^31)");
        if ((rc = fetch(col_idx, hrp[m], true, hci)) != LP_OK) return rc;
        if ((rc = fetch(val, hrp[m], true, hval)) != LP_OK) return rc;
        if ((rc = fetch(b, m, true, hb)) != LP_OK) return rc;
        if ((rc = fetch(c, n, true, hc)) != LP_OK) return rc;
        row_ptr = hrp.data();
        col_idx = hci.data();
        val = hval.data();
        b = hb.data();
        c = hc.data();
    }
    rc = validate(m, n, nnz, row_ptr, col_idx, val);
    if (rc != LP_OK) return rc;
    if ((rc = check_vec(b, m, "b")) != LP_OK) return rc;
    if ((rc = check_vec(c, n, "c")) != LP_OK) return rc;
    if (!dev && (rc = check_device()) != LP_OK) return rc;
    lp_problem* p = new (std::nothrow) lp_problem();
    if (!p) return fail(LP_ENOMEM, "host allocation failed");
    p->m = m;
    p->n = n;
    p->nnz = nnz;
    p->opt = opt;
    p->dense = dense;
    // a dense A runs NE-SOR as SOR on the Gram matrix (the same iteration in exact arithmetic)
    p->gsor = dense && (opt.inner == LP_NESOR || opt.inner == LP_GSOR);
    if (p->gsor && m > 8192) {
        delete p;
        return fail(LP_ETOOBIG, "the Gram-matrix path needs m <= 8192");
    }
    p->st = (hipStream_t)opt.stream;
    (void)hipGetDevice(&p->device);
    rc = setup(p, row_ptr, col_idx, val, b, c);
    if (rc != LP_OK) {
        destroy(p);
        return rc;
    }
    *out = p;
    return LP_OK;
}

}  // extern "C"

extern "C" {

lp_status lp_create(int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                    const int32_t* col_idx, const double* val, const double* b, const double* c,
                    const lp_options* o, lp_problem** out) {
    return create_impl(m, n, nnz, row_ptr, col_idx, val, b, c, o, false, out);
}

lp_status lp_create_bounded(int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                            const int32_t* col_idx, const double* val, const double* b, const double* c,
                            const double* lo, const double* hi, const lp_options* o, lp_problem** out) {
    g_err.clear();
    if (!out) return fail(LP_EINVAL, "NULL out");
    *out = nullptr;
    if (m < 1 || n < 1) return fail(LP_EDIM, "m and n must be positive");
    if (!row_ptr || !col_idx || !val || !b || !c || !lo || !hi) return fail(LP_EINVAL, "NULL input array");
    lp_options opt;
    if (o) opt = *o;
    else lp_options_default(&opt);
    lp_status rc = check_options(opt, false);
    if (rc != LP_OK) return rc;
    std::vector<int64_t> hrp;
    std::vector<int32_t> hci;
    std::vector<double> hval, hb, hc, hlo, hhi;
    if (opt.device_io) {
        if ((rc = check_device()) != LP_OK) return rc;
        if ((rc = fetch(row_ptr, m + 1, true, hrp)) != LP_OK) return rc;
        if (hrp[m] < 1 || hrp[m] >= ((int64_t)1 << 31)) return fail(LP_EDIM, "nnz must be in [1, 2^31)");
        if ((rc = fetch(col_idx, hrp[m], true, hci)) != LP_OK) return rc;
        if ((rc = fetch(val, hrp[m], true, hval)) != LP_OK) return rc;
        if ((rc = fetch(b, m, true, hb)) != LP_OK) return rc;
        if ((rc = fetch(c, n, true, hc)) != LP_OK) return rc;
        if ((rc = fetch(lo, n, true, hlo)) != LP_OK) return rc;
        if ((rc = fetch(hi, n, true, hhi)) != LP_OK) return rc;
        row_ptr = hrp.data();
        col_idx = hci.data();
        val = hval.data();
        b = hb.data();
        c = hc.data();
        lo = hlo.data();
        hi = hhi.data();
    }
    if (row_ptr[m] != nnz) return fail(LP_EINVAL, "row_ptr must end at nnz");
    StdForm sf;
    auto bm = std::make_unique<BoundMap>();
    if ((rc = bounded_standard(m, n, row_ptr, col_idx, val, b, c, lo, hi, sf, *bm)) != LP_OK) return rc;
    rc = create_impl(sf.m, sf.n, sf.rp.back(), sf.rp.data(), sf.ci.data(), sf.val.data(), sf.b.data(),
                     sf.c.data(), &opt, false, out, true);
    if (rc != LP_OK) return rc;
    lp_problem* p = *out;
    // the split free variables' column pairs, recentred by the interior-point steps
    std::vector<int32_t> pairs;
    for (int64_t j = 0; j < bm->n0; ++j)
        if (bm->kind[(size_t)j] == BK_FREE) {
            pairs.push_back((int32_t)bm->col[(size_t)j]);
            pairs.push_back((int32_t)bm->col2[(size_t)j]);
        }
    if (!pairs.empty()) {
        p->nfpairs = (int32_t)(pairs.size() / 2);
        p->fpairs = p->arena.alloc<int32_t>((int64_t)pairs.size());
        if (!p->fpairs) {
            destroy(p);
            *out = nullptr;
            return fail(LP_ENOMEM, "device allocation failed");
        }
        hipError_t e = hipMemcpy(p->fpairs, pairs.data(), sizeof(int32_t) * pairs.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            destroy(p);
            *out = nullptr;
            return hip_fail(e, "hipMemcpy");
        }
    }
    p->bounds = std::move(bm);
    return LP_OK;
}

lp_status lp_bounded_solution(const lp_problem* pc, double* x, double* y, double* obj) {
    g_err.clear();
    lp_problem* p = const_cast<lp_problem*>(pc);
    if (!p) return fail(LP_EINVAL, "NULL problem");
    if (!p->bounds) return fail(LP_EINVAL, "the problem was not created by lp_create_bounded");
    const BoundMap& bm = *p->bounds;
    std::vector<double> xs((size_t)p->n), ys((size_t)p->m), xo((size_t)bm.n0);
    LPK_HIP(hipMemcpyAsync(xs.data(), p->vec[V_X], sizeof(double) * p->n, hipMemcpyDeviceToHost, p->st));
    scatter(p->st, p->m, p->vec[V_Y], p->perm_d, p->vec[V_TMPM]);
    LPK_HIP(hipMemcpyAsync(ys.data(), p->vec[V_TMPM], sizeof(double) * p->m, hipMemcpyDeviceToHost, p->st));
    LPK_HIP(hipStreamSynchronize(p->st));
    bounds_recover(bm, xs.data(), xo.data());
    if (obj) {
        double s = 0.0;
        for (int64_t j = 0; j < bm.n0; ++j) s += bm.c0[(size_t)j] * xo[(size_t)j];
        *obj = s;
    }
    if (p->opt.device_io) {
        if (x) LPK_HIP(hipMemcpyAsync(x, xo.data(), sizeof(double) * bm.n0, hipMemcpyHostToDevice, p->st));
        if (y) LPK_HIP(hipMemcpyAsync(y, ys.data(), sizeof(double) * bm.m0, hipMemcpyHostToDevice, p->st));
        LPK_HIP(hipStreamSynchronize(p->st));
    } else {
        if (x) memcpy(x, xo.data(), sizeof(double) * bm.n0);
        if (y) memcpy(y, ys.data(), sizeof(double) * bm.m0);
    }
    return LP_OK;
}

lp_status lp_create_dense(int64_t m, int64_t n, const double* A, int64_t lda, const double* b,
                          const double* c, const lp_options* o, lp_problem** out) {
    g_err.clear();
    if (!out) return fail(LP_EINVAL, "NULL out");
    *out = nullptr;
    if (m < 1 || n < 1) return fail(LP_EDIM, "m and n must be positive");
    if (m > n) return fail(LP_EDIM, "m > n: the problem statement assumes m <= n");
    if (lda < n) return fail(LP_EINVAL, "lda < n");
    if (!A || !b || !c) return fail(LP_EINVAL, "NULL input array");
    if (m * n >= ((int64_t)1 << 31)) return fail(LP_EDIM, "m * n must be below 2^31");
    lp_options opt;
    if (o) opt = *o;
    else lp_options_default(&opt);
    const bool dev = opt.device_io != 0;
    std::vector<double> hA;
    std::vector<double> hb, hc;
    lp_status rc;
    if (dev) {
        if ((rc = check_device()) != LP_OK) return rc;
        hA.resize((size_t)(m * lda));
        LPK_HIP(hipMemcpy(hA.data(), A, sizeof(double) * m * lda, hipMemcpyDeviceToHost));
        if ((rc = fetch(b, m, true, hb)) != LP_OK) return rc;
        if ((rc = fetch(c, n, true, hc)) != LP_OK) return rc;
        A = hA.data();
        b = hb.data();
        c = hc.data();
    }
    // every entry is kept, zero or not: the dense matrix as a full CSR
    std::vector<int64_t> rp((size_t)m + 1);
    std::vector<int32_t> ci((size_t)(m * n));
    std::vector<double> val((size_t)(m * n));
    for (int64_t i = 0; i < m; ++i) {
        rp[i] = i * n;
        for (int64_t j = 0; j < n; ++j) {
            ci[i * n + j] = (int32_t)j;
            val[i * n + j] = A[i * lda + j];
        }
    }
    rp[m] = m * n;
    lp_options o2 = opt;
    o2.device_io = 0;
    rc = create_impl(m, n, m * n, rp.data(), ci.data(), val.data(), b, c, &o2, true, out);
    if (rc == LP_OK) (*out)->opt.device_io = opt.device_io;
    return rc;
}

void lp_destroy(lp_problem* p) { destroy(p); }

// run the problem alone (its batch of one) until it leaves the engine, or (one_step) until
// it has taken one interior-point step
static lp_status run_solo(lp_problem* p, bool from_point, int32_t limit_k, bool one_step, Engine::Member* out) {
    Batch* b = nullptr;
    lp_status rc = solo_batch(p, &b);
    if (rc != LP_OK) return rc;
    Engine E;
    E.attach(b);
    E.stepwise = one_step;
    const int s = E.join(p, from_point, limit_k);
    if (s < 0) return fail(LP_EINVAL, "no slot");
    while (E.any_live()) {
        if (one_step && E.mem[s].steps > 0) break;
        rc = E.round();
        if (rc != LP_OK) return rc;
    }
    *out = E.mem[s];
    return LP_OK;
}

lp_status ipm_step(lp_problem* p, lp_iter_info* info) {
    g_err.clear();
    if (!p) return fail(LP_EINVAL, "NULL problem");
    if (!p->have_point && p->opt.start != 0) return fail(LP_EINVAL, "start == 1 needs lp_set_state first");
    Engine::Member mb;
    // without a point, the starting point comes first, then the step
    lp_status rc = run_solo(p, p->have_point, INT32_MAX, true, &mb);
    if (rc != LP_OK) return rc;
    if (info) *info = mb.L;
    return mb.state == Engine::DONE && mb.status == LP_DIVERGED ? LP_DIVERGED : LP_OK;
}

lp_status lp_solve(lp_problem* p, lp_result* r) {
    g_err.clear();
    if (!p) return fail(LP_EINVAL, "NULL problem");
    const double t0 = now_seconds();
    p->log.clear();
    p->krylov_total = 0;
    bool from_point = false;
    if (p->opt.start != 0) {
        if (!p->have_point) return fail(LP_EINVAL, "start == 1 needs lp_set_state first");
        p->ist.eps_in = p->opt.eps_in0;
        p->ist.k = 0;
        p->ist.fail_prev = 0;
        from_point = true;
    }
    Engine::Member mb;
    lp_status rc = run_solo(p, from_point, p->opt.ipm_max_iter, false, &mb);
    if (rc != LP_OK) return rc;
    if (r) {
        fill_result(mb, r);
        r->seconds = now_seconds() - t0;
    }
    return mb.status;
}

lp_status direction_solve(lp_problem* p, const double* d, const double* f, double tol, double* dw,
                          double* dy, lp_krylov_info* ki) {
    g_err.clear();
    if (!p) return fail(LP_EINVAL, "NULL problem");
    if (!f || !dw) return fail(LP_EINVAL, "NULL f or dw");
    if (!(tol >= 0.0)) return fail(LP_EINVAL, "tol must be >= 0");
    const int64_t m = p->m, n = p->n;
    lp_status rc;
    if (!p->opt.device_io) {
        if ((rc = check_vec(f, m, "f")) != LP_OK) return rc;
        if (d) {
            if ((rc = check_vec(d, n, "d")) != LP_OK) return rc;
            for (int64_t j = 0; j < n; ++j)
                if (!(d[j] > 0.0)) return fail(LP_EINVAL, "d must be positive");
        }
    }
    if (!d && !p->have_point) return fail(LP_EINVAL, "no current iterate: pass d");
    Batch* b = nullptr;
    if ((rc = solo_batch(p, &b)) != LP_OK) return rc;
    hipStream_t st = b->st;
    Param& pr = b->h_param[0];
    if (d) {
        if ((rc = copy_in(p, d, p->vec[V_D], n)) != LP_OK) return rc;
    } else {
        // D = diag(sqrt(x/s)) of the current iterate
        pr.mode = MD_RUN | MD_SCALE;
        if ((rc = b->put_params()) != LP_OK) return rc;
        b_scaling(b->L);
        LPK_HIP(hipStreamSynchronize(st));   // the parameters are written again below
    }
    pr.mode = MD_API;
    pr.scal[SC_TOL] = tol;
    if (p->opt.inner == LP_CIMMINO && !p->gsor) {
        if (p->opt.omega_c > 0.0) pr.scal[SC_OMC] = p->opt.omega_c;
        else pr.mode |= MD_POW;
    }
    if ((rc = b->put_params()) != LP_OK) return rc;
    if ((rc = scale_batch(*b, MD_API)) != LP_OK) return rc;
    if ((rc = copy_in(p, f, p->vec[V_TMPM], m)) != LP_OK) return rc;
    gather(st, m, p->vec[V_TMPM], p->perm_d, p->vec[V_F]);
    std::vector<lp_krylov_info> info;
    if ((rc = krylov_batch(*b, MD_API, &info)) != LP_OK) return rc;
    if (ki) *ki = info[0];
    if ((rc = copy_out(p, p->vec[V_DW], dw, n)) != LP_OK) return rc;
    if (dy) {
        b_div_rho(b->L, V_DYC, V_DYH, MD_API);
        scatter(st, m, p->vec[V_DYC], p->perm_d, p->vec[V_TMPM]);
        if ((rc = copy_out(p, p->vec[V_TMPM], dy, m)) != LP_OK) return rc;
    }
    LPK_HIP(hipGetLastError());
    LPK_HIP(hipStreamSynchronize(st));
    return LP_OK;
}

lp_status lp_get_state(const lp_problem* pc, double* x, double* y, double* s, lp_ipm_state* stt) {
    g_err.clear();
    lp_problem* p = const_cast<lp_problem*>(pc);
    if (!p) return fail(LP_EINVAL, "NULL problem");
    lp_status rc;
    if (x && (rc = copy_out(p, p->vec[V_X], x, p->n)) != LP_OK) return rc;
    if (s && (rc = copy_out(p, p->vec[V_S], s, p->n)) != LP_OK) return rc;
    if (y) {
        scatter(p->st, p->m, p->vec[V_Y], p->perm_d, p->vec[V_TMPM]);
        if ((rc = copy_out(p, p->vec[V_TMPM], y, p->m)) != LP_OK) return rc;
    }
    LPK_HIP(hipStreamSynchronize(p->st));
    if (stt) *stt = p->ist;
    return LP_OK;
}

lp_status lp_set_state(lp_problem* p, const double* x, const double* y, const double* s,
                       const lp_ipm_state* stt) {
    g_err.clear();
    if (!p) return fail(LP_EINVAL, "NULL problem");
    if (!x || !y || !s) return fail(LP_EINVAL, "NULL x, y or s");
    lp_status rc;
    if (!p->opt.device_io) {
        if ((rc = check_vec(x, p->n, "x")) != LP_OK) return rc;
        if ((rc = check_vec(s, p->n, "s")) != LP_OK) return rc;
        if ((rc = check_vec(y, p->m, "y")) != LP_OK) return rc;
        for (int64_t j = 0; j < p->n; ++j)
            if (!(x[j] > 0.0) || !(s[j] > 0.0)) return fail(LP_EINVAL, "x and s must be positive");
    }
    if ((rc = copy_in(p, x, p->vec[V_X], p->n)) != LP_OK) return rc;
    if ((rc = copy_in(p, s, p->vec[V_S], p->n)) != LP_OK) return rc;
    if ((rc = copy_in(p, y, p->vec[V_TMPM], p->m)) != LP_OK) return rc;
    gather(p->st, p->m, p->vec[V_TMPM], p->perm_d, p->vec[V_Y]);
    if (p->opt.device_io) {
        Batch* b = nullptr;
        if ((rc = solo_batch(p, &b)) != LP_OK) return rc;
        b->h_param[0].mode = MD_API;
        if ((rc = b->put_params()) != LP_OK) return rc;
        b_min2(b->L, MD_API);
        const int ops[2] = {1, 1};
        b_red_finish(b->L, 2, ops, MD_API, 0);
        LPK_HIP(hipGetLastError());
        if ((rc = b->get_slots()) != LP_OK) return rc;
        const double* q = b->h_slot[0].out;
        if (!(q[0] > 0.0) || !(q[1] > 0.0)) return fail(LP_EINVAL, "x and s must be positive");
    }
    LPK_HIP(hipStreamSynchronize(p->st));
    if (stt) {
        p->ist = *stt;
    } else {
        p->ist.eps_in = p->opt.eps_in0;
        p->ist.k = 0;
        p->ist.fail_prev = 0;
    }
    p->have_point = true;
    return LP_OK;
}

lp_status lp_get_log(const lp_problem* p, lp_iter_info* info, int32_t cap, int32_t* n_out) {
    if (!p || !n_out) return fail(LP_EINVAL, "NULL argument");
    const int32_t cnt = (int32_t)p->log.size();
    *n_out = cnt;
    if (info)
        for (int32_t i = 0; i < cnt && i < cap; ++i) info[i] = p->log[i];
    return LP_OK;
}

lp_status lp_footprint_bytes(int64_t m, int64_t n, int64_t nnz, const lp_options* o, uint64_t* bytes) {
    if (!bytes) return fail(LP_EINVAL, "NULL bytes");
    if (m < 1 || n < 1 || m > n || nnz < 1 || nnz >= ((int64_t)1 << 31)) return fail(LP_EDIM, "bad dimensions");
    lp_options opt;
    if (o) opt = *o;
    else lp_options_default(&opt);
    *bytes = footprint(m, n, nnz, opt);
    return LP_OK;
}

lp_status lp_sweep_layout(const lp_problem* p, int32_t* fp32, int32_t* kind) {
    if (!p) return fail(LP_EINVAL, "NULL problem");
    if (fp32) *fp32 = p->mixed ? 1 : 0;
    if (kind) *kind = p->lds_kind;
    return LP_OK;
}

lp_status lp_colouring(const lp_problem* p, int32_t* ncolours, int32_t* sizes, int32_t cap) {
    if (!p || !ncolours) return fail(LP_EINVAL, "NULL argument");
    *ncolours = (int32_t)p->colours.size();
    if (sizes)
        for (int32_t c = 0; c < *ncolours && c < cap; ++c) sizes[c] = p->colours[c].r1 - p->colours[c].r0;
    return LP_OK;
}

lp_status lp_bounds_standard_form(int64_t m, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                                  const double* val, const double* b, const double* c, const double* lo,
                                  const double* hi, int64_t* m_out, int64_t* n_out, int64_t* nnz_out,
                                  int64_t* row_ptr_out, int32_t* col_idx_out, double* val_out, double* b_out,
                                  double* c_out, double* offset) {
    g_err.clear();
    if (!m_out || !n_out || !nnz_out) return fail(LP_EINVAL, "NULL size output");
    if (!row_ptr) return fail(LP_EINVAL, "NULL input array");
    StdForm sf;
    BoundMap bm;
    lp_status rc = bounded_standard(m, n, row_ptr, col_idx, val, b, c, lo, hi, sf, bm);
    if (rc != LP_OK) return rc;
    *m_out = sf.m;
    *n_out = sf.n;
    *nnz_out = sf.rp.back();
    if (!row_ptr_out) return LP_OK;   // size query
    if (!col_idx_out || !val_out || !b_out || !c_out) return fail(LP_EINVAL, "NULL output array");
    std::copy(sf.rp.begin(), sf.rp.end(), row_ptr_out);
    std::copy(sf.ci.begin(), sf.ci.end(), col_idx_out);
    std::copy(sf.val.begin(), sf.val.end(), val_out);
    std::copy(sf.b.begin(), sf.b.end(), b_out);
    std::copy(sf.c.begin(), sf.c.end(), c_out);
    if (offset) *offset = bm.offset;
    return LP_OK;
}

lp_status lp_presolve_rows(int64_t m, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                           const double* val, const double* b, double tol, int32_t* keep, int64_t* m_keep) {
    g_err.clear();
    if (!row_ptr || !col_idx || !val || !b || !keep || !m_keep) return fail(LP_EINVAL, "NULL argument");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(LP_EINVAL, "tol must be finite and >= 0");
    if (m < 1 || n < 1) return fail(LP_EDIM, "m and n must be positive");
    lp_status rc = validate(m, n, row_ptr[m], row_ptr, col_idx, val, false);
    if (rc != LP_OK) return rc;
    if ((rc = check_vec(b, m, "b")) != LP_OK) return rc;
    std::string err;
    if (!presolve_parallel_rows(m, row_ptr, col_idx, val, b, tol, keep, m_keep, err)) return fail(LP_EINVAL, err);
    return LP_OK;
}

// rows up to which the dependency search may fall back to the dense Gram matrix (8 m^2
// bytes, m^3 / 3 multiply-adds)
static constexpr int64_t PRESOLVE_GRAM_MAX_M = 4096;

lp_status lp_presolve_dependent_rows(int64_t m, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                                     const double* val, const double* b, double tol, int32_t* keep,
                                     int64_t* m_keep) {
    g_err.clear();
    if (!row_ptr || !col_idx || !val || !b || !keep || !m_keep) return fail(LP_EINVAL, "NULL argument");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(LP_EINVAL, "tol must be finite and >= 0");
    if (m < 1 || n < 1) return fail(LP_EDIM, "m and n must be positive");
    lp_status rc = validate(m, n, row_ptr[m], row_ptr, col_idx, val, false);
    if (rc != LP_OK) return rc;
    if ((rc = check_vec(b, m, "b")) != LP_OK) return rc;
    std::string err;
    const int64_t max_fill = std::max<int64_t>(32 * row_ptr[m], (int64_t)1 << 22);
    try {
        if (presolve_dependent_rows(m, n, row_ptr, col_idx, val, b, tol, max_fill, keep, m_keep, err)) return LP_OK;
        if (err.find("fill limit") == std::string::npos) return fail(LP_EINVAL, err);
        // the elimination filled: the dense Gram matrix, where it fits
        if (m > PRESOLVE_GRAM_MAX_M)
            return fail(LP_ETOOBIG, err + ", and m exceeds the dense fallback's " +
                                        std::to_string(PRESOLVE_GRAM_MAX_M) + " rows");
        err.clear();
        if (presolve_dependent_rows_gram(m, n, row_ptr, col_idx, val, b, tol, keep, m_keep, err)) return LP_OK;
        return fail(LP_EINVAL, err);
    } catch (const std::bad_alloc&) {
        return fail(LP_ENOMEM, "host memory for the dependency search");
    }
}

lp_status lp_colour_rows(int64_t m, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                         int32_t* colour, int32_t* perm, int32_t* ncolours) {
    g_err.clear();
    if (!row_ptr || !col_idx || !colour || !perm || !ncolours) return fail(LP_EINVAL, "NULL argument");
    if (m < 1 || n < 1) return fail(LP_EDIM, "m and n must be positive");
    if (row_ptr[0] != 0) return fail(LP_EINVAL, "row_ptr[0] != 0");
    for (int64_t i = 0; i < m; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return fail(LP_EINVAL, "row_ptr decreasing");
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col_idx[k] < 0 || col_idx[k] >= n) return fail(LP_EINVAL, "column index out of range");
    }
    *ncolours = greedy_colour(m, n, row_ptr, col_idx, colour, perm);
    return LP_OK;
}

const char* lp_status_str(lp_status s) {
    switch (s) {
        case LP_OK: return "LP_OK";
        case LP_EINVAL: return "LP_EINVAL";
        case LP_EDIM: return "LP_EDIM";
        case LP_ENONFINITE: return "LP_ENONFINITE";
        case LP_ENOMEM: return "LP_ENOMEM";
        case LP_ETOOBIG: return "LP_ETOOBIG";
        case LP_EDEVICE: return "LP_EDEVICE";
        case LP_NOT_CONVERGED: return "LP_NOT_CONVERGED";
        case LP_DIVERGED: return "LP_DIVERGED";
        case LP_KRYLOV_MAXIT: return "LP_KRYLOV_MAXIT";
    }
    return "LP_UNKNOWN";
}

const char* lp_last_error(void) { return g_err.c_str(); }

const char* lp_version(void) { return "lpk 0.1 (gfx950)"; }

}  // extern "C"
