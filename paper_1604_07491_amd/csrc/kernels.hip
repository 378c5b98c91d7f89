// Batched HIP kernels of the interior-point direction path for CDNA4 (gfx950, wave64).
//
// Grid (x, S): one row of blocks per instance (see block_map), Inst[instance] its descriptor.  Reductions
// are two-stage (per-block partials, then one fixed-order pass per instance), so results
// are deterministic and do not depend on the other instances of the batch.
//
// Layout (per instance):
//  * A is held row-permuted into colour-major order (rows of one colour contiguous) as CSR
//    with int32 row pointers and column indices; the CSC copy indexes the permuted rows.
//  * A_hat = diag(rho)^-1 A D (unit rows, Sec. 3.5) is materialised once per scaling in
//    both layouts (FP64) and, in mixed precision, as FP32 copies.
//  * The Krylov basis V and the multiplier vectors P are column-major m x (kmax+1).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.h"
#include "kernel_util.h"

namespace lpk {

int red_blocks(int64_t len) {
    int64_t b = (len + BLOCK * 4 - 1) / (BLOCK * 4);
    if (b < 1) b = 1;
    if (b > RED_MAXBLK) b = RED_MAXBLK;
    return (int)b;
}

int spmv_blocks(int64_t rows, int g) { return (int)capg(cdiv(rows * g, BLOCK), RED_MAXBLK); }

// ------------------------------------------------------------------------------------
// row-dot products: out[r] = epi(sum_k val[k] x[idx[k]]), one sub-group of g lanes per row,
// grid-stride over the rows of the instance
__global__ __launch_bounds__(BLOCK) void k_spmv(const Inst* __restrict__ I, int mat, int xsel,
                                                int outsel, int epi, int b1sel, int b2sel,
                                                int pmask, int nrm) {
    __shared__ double sh[BLOCK / 64];
    INST;
    if (!takes_part(in, pmask)) return;
    int rows, g;
    const int32_t *ptr, *idx;
    const double* val;
    if (mat == M_A_CSR || mat == M_AH_CSR) {
        rows = in.m; g = in.g_csr; ptr = in.rp; idx = in.ci; val = mat == M_A_CSR ? in.a : in.ah;
    } else {
        rows = in.n; g = in.g_csc; ptr = in.cp; idx = in.ri; val = mat == M_A_CSC ? in.ac : in.ahc;
    }
    const int64_t kcol = xsel < 0 ? (int64_t)to_global(in.ctl)->k * in.ldv : 0;
    const LPK_GLOBAL double* __restrict__ x =
        to_global(xsel == V_PCOL ? in.P + kcol : xsel == V_VCOL ? in.V + kcol : in.vec[xsel]);
    LPK_GLOBAL double* __restrict__ out = to_global(in.vec[outsel]);
    const LPK_GLOBAL double* __restrict__ b1 = to_global(b1sel >= 0 ? in.vec[b1sel] : nullptr);
    const LPK_GLOBAL double* __restrict__ b2 = to_global(b2sel >= 0 ? in.vec[b2sel] : nullptr);
    const LPK_GLOBAL int32_t* __restrict__ gptr = to_global(ptr);
    const int lane = threadIdx.x & (g - 1);
    const int lg = __ffs(g) - 1;   // g is a power of two
    const int64_t total = (int64_t)rows * g;
    // the reduction's partition depends on the instance alone (nbs blocks)
    const int nb = nrm ? in.nbs : (int)gridDim.x;
    if (bx >= nb) return;
    double q = 0.0;
    for (int64_t t0 = (int64_t)bx * BLOCK; t0 < total; t0 += (int64_t)nb * BLOCK) {
        const int64_t t = t0 + threadIdx.x;
        const int row = (int)(t >> lg);
        double sum = 0.0;
        if (row < rows) {
            const int s = gptr[row], e = gptr[row + 1];
            sum = row_dot<8>(to_global(val), to_global(idx), x, s, e, lane, g);
        }
        sum = sg_sum(sum, g);
        if (row < rows && lane == 0) {
            double o;
            if (epi == EPI_B_MINUS) o = b1[row] - sum;
            else if (epi == EPI_B1_MINUS_B2) o = b1[row] - sum - b2[row];
            else if (epi == EPI_B_PLUS) o = b1[row] + sum;
            else o = sum;
            out[row] = o;
            q += o * o;
        }
    }
    if (nrm) {
        const double r = block_sum(q, sh);
        write_part(in, bx, 0, r);
    }
}

// ------------------------------------------------------------------------------------
// out = A_hat x for instances with sliced colours: blocks [0, nbc) take the rows kept in
// CSR form (g_csr lanes per row, grid-stride over their list), block nbc + q takes
// slice q as the sliced sweep does (thread: row r = lane mod SL_ROWS, slots
// 4 w + lane / SL_ROWS + SL_GROUPS t; the four slot groups of a wave by two butterfly
// steps, then the waves in order).  Instances without slices take the plain row-dot form.
__global__ __launch_bounds__(SL_THREADS) void k_spmv_ahz(const Inst* __restrict__ I, int xsel, int outsel, int pmask) {
    __shared__ double red[SL_THREADS / 64][SL_ROWS];
    INST;
    if (!takes_part(in, pmask)) return;
    const int64_t kcol = xsel < 0 ? (int64_t)to_global(in.ctl)->k * in.ldv : 0;
    const LPK_GLOBAL double* __restrict__ x =
        to_global(xsel == V_PCOL ? in.P + kcol : xsel == V_VCOL ? in.V + kcol : in.vec[xsel]);
    LPK_GLOBAL double* __restrict__ out = to_global(in.vec[outsel]);
    const int nbc = in.nsl > 0 ? in.nbc : (int)gridDim.x;
    if (bx < nbc) {
        const int g = in.g_csr;
        const int lane = threadIdx.x & (g - 1);
        const int lg = __ffs(g) - 1;
        // with slices, the listed CSR rows; else every row
        const LPK_GLOBAL int32_t* __restrict__ crow = to_global(in.nsl > 0 ? in.crow : nullptr);
        const int rows = crow ? in.ncrow : in.m;
        const int64_t total = (int64_t)rows * g;
        const LPK_GLOBAL int32_t* __restrict__ rp = to_global(in.rp);
        for (int64_t t0 = (int64_t)bx * SL_THREADS; t0 < total; t0 += (int64_t)nbc * SL_THREADS) {
            const int q = (int)((t0 + threadIdx.x) >> lg);
            const bool mine = q < rows;
            const int row = mine ? (crow ? crow[q] : q) : 0;
            double sum = 0.0;
            if (mine) sum = row_dot<8>(to_global((const double*)in.ah), to_global(in.ci), x, rp[row], rp[row + 1], lane, g);
            sum = sg_sum(sum, g);
            if (mine && lane == 0) out[row] = sum;
        }
        return;
    }
    const int q = bx - nbc;
    if (q >= in.nsl) return;   // the same for the whole block
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int r = ln & (SL_ROWS - 1);
    const int grp = wv * (64 / SL_ROWS) + ln / SL_ROWS;
    const int off = to_global(in.soff)[q];
    const int steps = to_global(in.slen)[q] / SL_GROUPS;
    const LPK_GLOBAL double* __restrict__ val = to_global((const double*)in.sl_val);
    const LPK_GLOBAL int32_t* __restrict__ idx = to_global(in.sl_idx);
    const int base = off + grp * SL_ROWS + r;
    constexpr int STEP = SL_GROUPS * SL_ROWS;
    // up to 12 slot steps at a time (a transportation sink slice has 10): all their loads,
    // then all their gathers
    double acc = 0.0;
    for (int t0 = 0; t0 < steps; t0 += 12) {
        double v[12], xv[12];
        int j[12];
#pragma unroll
        for (int u = 0; u < 12; ++u) {
            const bool ok = t0 + u < steps;
            j[u] = ok ? idx[base + (t0 + u) * STEP] : -1;
            v[u] = ok ? val[base + (t0 + u) * STEP] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 12; ++u) xv[u] = j[u] >= 0 ? x[j[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < 12; ++u) acc += v[u] * xv[u];
    }
    acc += __shfl_xor(acc, 16, 64);
    acc += __shfl_xor(acc, 32, 64);
    if (ln < SL_ROWS) red[wv][ln] = acc;
    __syncthreads();
    if (wv == 0 && ln < SL_ROWS) {
        const LPK_GLOBAL int32_t* sr = to_global(in.srows) + 2 * q;
        if (r < sr[1]) {
            double tot = 0.0;
#pragma unroll
            for (int w = 0; w < SL_THREADS / 64; ++w) tot += red[w][r];
            out[sr[0] + r] = tot;
        }
    }
}

void b_spmv(const BLaunch& L, int mat, int xsel, int outsel, int epi, int b1sel, int b2sel, int pmask,
            bool nrm) {
    if (mat == M_AH_CSR && epi == EPI_PLAIN && !nrm && L.grid_ahz > 0) {
        hipLaunchKernelGGL(k_spmv_ahz, dim3(capg(L.grid_ahz, 1 << 30), L.S), dim3(SL_THREADS), 0, L.st, L.I, xsel, outsel,
                           pmask);
        return;
    }
    const unsigned gx = nrm ? (unsigned)L.max_nbs : capg(L.grid_spmv[mat], GRID_CAP);
    hipLaunchKernelGGL(k_spmv, dim3(gx, L.S), dim3(BLOCK), 0, L.st, L.I, mat, xsel, outsel, epi, b1sel,
                       b2sel, pmask, nrm ? 1 : 0);
}

// ------------------------------------------------------------------------------------
// Cimmino inner iterations: r = v - A_hat z (first sweep: z = 0, r = v); p += w r;
// z (+)= w A_hat^T r.  w = ctl->omega_c.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cim_res(const Inst* __restrict__ I, int first) {
    INST;
    if (in.ctl->done || in.gsor || other_precision<T>(in)) return;
    const int g = in.g_csr;
    const int lane = threadIdx.x & (g - 1);
    const int64_t k = in.ctl->k;
    const T* __restrict__ val;
    const T* __restrict__ z;
    T* __restrict__ r;
    if constexpr (sizeof(T) == 4) {
        val = (const T*)in.ah32; z = (const T*)in.z32; r = (T*)in.r32;
    } else {
        val = (const T*)in.ah; z = (const T*)in.vec[V_Z64]; r = (T*)in.vec[V_R64];
    }
    const double w = in.ctl->omega_c;
    const int64_t total = (int64_t)in.m * g;
    for (int64_t t0 = (int64_t)bx * BLOCK; t0 < total; t0 += (int64_t)gridDim.x * BLOCK) {
        const int64_t t = t0 + threadIdx.x;
        const int row = (int)(t / g);
        T sum = 0;
        if (!first && row < in.m) {
            const int s = in.rp[row], e = in.rp[row + 1];
            for (int kk = s + lane; kk < e; kk += g) sum += val[kk] * z[in.ci[kk]];
        }
        if (!first) sum = sg_sum(sum, g);
        if (row < in.m && lane == 0) {
            double vrow;
            if (first) {
                // first sweep: v_k = u / h_{k,k-1} is formed here and stored
                vrow = in.vec[V_U][row] * in.ctl->inv_h;
                in.V[k * in.ldv + row] = vrow;
            } else {
                vrow = in.V[k * in.ldv + row];
            }
            const T rr = (T)vrow - sum;
            r[row] = rr;
            if (first) in.P[k * in.ldv + row] = w * (double)rr;
            else in.P[k * in.ldv + row] += w * (double)rr;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cim_z(const Inst* __restrict__ I, int first) {
    INST;
    if (in.ctl->done || in.gsor || other_precision<T>(in)) return;
    const int g = in.g_csc;
    const int lane = threadIdx.x & (g - 1);
    const T* __restrict__ cval;
    const T* __restrict__ r;
    T* __restrict__ z;
    if constexpr (sizeof(T) == 4) {
        cval = (const T*)in.ahc32; r = (const T*)in.r32; z = (T*)in.z32;
    } else {
        cval = (const T*)in.ahc; r = (const T*)in.vec[V_R64]; z = (T*)in.vec[V_Z64];
    }
    const T wc = (T)in.ctl->omega_c;
    const int64_t total = (int64_t)in.n * g;
    for (int64_t t0 = (int64_t)bx * BLOCK; t0 < total; t0 += (int64_t)gridDim.x * BLOCK) {
        const int64_t t = t0 + threadIdx.x;
        const int col = (int)(t / g);
        T sum = 0;
        if (col < in.n) {
            const int s = in.cp[col], e = in.cp[col + 1];
            for (int kk = s + lane; kk < e; kk += g) sum += cval[kk] * r[in.ri[kk]];
        }
        sum = sg_sum(sum, g);
        if (col < in.n && lane == 0) z[col] = first ? wc * sum : z[col] + wc * sum;
    }
}

void b_cim_res(const BLaunch& L, int first) {
    const unsigned gx = capg(L.grid_spmv[M_AH_CSR], GRID_CAP);
    if (L.any32) hipLaunchKernelGGL((k_cim_res<float>), dim3(gx, L.S), dim3(BLOCK), 0, L.st, L.I, first);
    if (L.any64) hipLaunchKernelGGL((k_cim_res<double>), dim3(gx, L.S), dim3(BLOCK), 0, L.st, L.I, first);
}
void b_cim_z(const BLaunch& L, int first) {
    const unsigned gx = capg(L.grid_spmv[M_AH_CSC], GRID_CAP);
    if (L.any32) hipLaunchKernelGGL((k_cim_z<float>), dim3(gx, L.S), dim3(BLOCK), 0, L.st, L.I, first);
    if (L.any64) hipLaunchKernelGGL((k_cim_z<double>), dim3(gx, L.S), dim3(BLOCK), 0, L.st, L.I, first);
}

// ------------------------------------------------------------------------------------
// Dense path: P[:,k] = C v_k (the inner-iteration preconditioner as a matrix) and the
// Krylov operator u = G p_k; one wave per row of the m x m row-major matrices
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_apply_c(const Inst* __restrict__ I) {
    INST;
    if (in.ctl->done || !in.gsor || other_precision<T>(in)) return;
    const int64_t k = in.ctl->k;
    const int m = in.m;
    const int i = bx * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= m) return;
    // v_k = u / h_{k,k-1} formed on the fly; row i stores its entry of V[:,k]
    const double* __restrict__ u = in.vec[V_U];
    const double ih = in.ctl->inv_h;
    const T* __restrict__ ci;
    if constexpr (sizeof(T) == 4) ci = (const T*)in.C32 + (int64_t)i * m;
    else ci = (const T*)in.C + (int64_t)i * m;
    if (lane == 0) in.V[k * in.ldv + i] = u[i] * ih;
    T acc = 0;
    for (int j = lane; j < m; j += 64) acc += ci[j] * (T)(u[j] * ih);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) in.P[k * in.ldv + i] = (double)acc;
}

__global__ __launch_bounds__(BLOCK) void k_gemv_col(const Inst* __restrict__ I) {
    INST;
    if (in.ctl->done || !in.gsor) return;
    const int m = in.m;
    const double* __restrict__ p = in.P + (int64_t)in.ctl->k * in.ldv;
    const int i = bx * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= m) return;
    const double* __restrict__ gi = in.G + (int64_t)i * m;
    double acc = 0.0;
    for (int j = lane; j < m; j += 64) acc += gi[j] * p[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) in.vec[V_U][i] = acc;
}

void b_apply_c(const BLaunch& L) {
    if (L.any32) hipLaunchKernelGGL((k_apply_c<float>), dim3(cdiv(L.max_m, 4), L.S), dim3(BLOCK), 0, L.st, L.I);
    if (L.any64) hipLaunchKernelGGL((k_apply_c<double>), dim3(cdiv(L.max_m, 4), L.S), dim3(BLOCK), 0, L.st, L.I);
}
void b_gemv_col(const BLaunch& L) {
    hipLaunchKernelGGL(k_gemv_col, dim3(cdiv(L.max_m, 4), L.S), dim3(BLOCK), 0, L.st, L.I);
}

// ------------------------------------------------------------------------------------
// Classical Gram-Schmidt applied twice on V (m x (k+1), column-major), in two kinds of
// launch per pass:
//  * dots: the dot products of u with the columns of V.  One wave computes the dot of a
//    whole segment of GS_SEG rows of one column (16 rows per lane, four independent
//    accumulators, one wave reduction) and writes it to part[segment][j]; with m <=
//    GS_SEG a dot is complete in one wave.  The waves of an instance loop over its
//    (column, segment) tasks.
//  * update: u -= V h by row chunks of 64 * RPL rows, the waves of a block splitting the
//    columns and adding their partial sums in LDS.  Fused: every block first sums the
//    segment partials of h itself (few segments, k + 1 <= GS_HLDS) and block 0 stores
//    (pass 0) or adds (pass 1) h in column k of H; otherwise k_gs_reduce does that first
//    and the update reads h from h2.  Pass 1 also writes the chunk's partial of ||u||^2.
// Buffers: pass 0 dots -> gpart, pass 1 dots -> gpart2, pass 1 norm partials -> gpart.
constexpr int GS_WAVES = 8;
constexpr int GS_HLDS = 2048;   // coefficients staged in LDS by the fused update
constexpr int GS_SEG = 1024;    // rows of one dot task
constexpr int GS_DOT_WAVES = 4; // waves per block of the dot launches (small blocks: the
                                // blocks beyond an instance's tasks cost less)

__global__ __launch_bounds__(64 * GS_DOT_WAVES) void k_gs_dots(const Inst* __restrict__ I, int pass) {
    INST;
    if (in.ctl->done) return;
    const int k = in.ctl->k;
    const int nseg = in.nseg;
    const int64_t m = in.m;
    const int tasks = nseg * (k + 1);   // < 2^31: nseg * (kmax + 1) doubles are allocated
    const int lane = threadIdx.x & 63;
    const int nw = (int)gridDim.x * GS_DOT_WAVES;
    const LPK_GLOBAL double* __restrict__ u = to_global(in.vec[V_U]);
    double* __restrict__ out = pass ? in.gpart2 : in.gpart;
    for (int t = bx * GS_DOT_WAVES + (threadIdx.x >> 6); t < tasks; t += nw) {
        const int j = nseg == 1 ? t : t / nseg;
        const int sg = t - j * nseg;
        const int64_t r0 = (int64_t)sg * GS_SEG;
        const int64_t r1 = r0 + GS_SEG < m ? r0 + GS_SEG : m;
        const LPK_GLOBAL double* __restrict__ vj = to_global(in.V + (int64_t)j * in.ldv);
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int64_t i = r0 + lane;
        for (; i + 192 < r1; i += 256) {
            a0 += vj[i] * u[i];
            a1 += vj[i + 64] * u[i + 64];
            a2 += vj[i + 128] * u[i + 128];
            a3 += vj[i + 192] * u[i + 192];
        }
        for (; i < r1; i += 64) a0 += vj[i] * u[i];
        const double a = wave_sum((a0 + a1) + (a2 + a3));
        if (lane == 0) out[(int64_t)sg * in.ldp + j] = a;
    }
}

// acc[t] += sum over the wave's columns j (w, w + GS_WAVES, ... <= k, increasing) of
// M[i_t, j] h[j], M column-major with the basis stride (V or P).  GS_U columns are loaded
// before any is used, so a wave keeps GS_U * RPL loads in flight; the order of every sum
// is that of the plain loop.
template <int RPL>
constexpr int gs_unroll() { return RPL >= 8 ? 1 : 8 / RPL; }

template <int RPL>
__device__ __forceinline__ void chunk_axpy(const Inst& in, const double* __restrict__ M, int k, int w, int lane,
                                           int64_t base, int rpl, const double* h, double (&acc)[RPL]) {
    constexpr int U = gs_unroll<RPL>();
    const int64_t m = in.m;
    int j = w;
    for (; j + (U - 1) * GS_WAVES <= k; j += U * GS_WAVES) {
        double v[U][RPL], hq[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            hq[q] = h[j + q * GS_WAVES];
            const LPK_GLOBAL double* __restrict__ vj = to_global(M + (int64_t)(j + q * GS_WAVES) * in.ldv);
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
                const int64_t i = base + lane + 64 * t;
                v[q][t] = (t < rpl && i < m) ? vj[i] : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
                const int64_t i = base + lane + 64 * t;
                if (t < rpl && i < m) acc[t] += v[q][t] * hq[q];
            }
    }
    for (; j <= k; j += GS_WAVES) {
        const double hj = h[j];
        const LPK_GLOBAL double* __restrict__ vj = to_global(M + (int64_t)j * in.ldv);
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int64_t i = base + lane + 64 * t;
            if (t < rpl && i < m) acc[t] += vj[i] * hj;
        }
    }
}

template <int RPL>
__global__ __launch_bounds__(64 * GS_WAVES) void k_gs_update(const Inst* __restrict__ I, int pass, int fused) {
    __shared__ double red[GS_WAVES][64 * RPL];
    __shared__ double sh[GS_WAVES];
    __shared__ double hl[GS_HLDS];
    INST;
    if (in.ctl->done || bx >= in.nchunks) return;
    const int k = in.ctl->k;
    const int rpl = in.rpl;   // <= RPL
    const int64_t m = in.m;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)bx * 64 * rpl;
    LPK_GLOBAL double* __restrict__ u = to_global(in.vec[V_U]);
    const double* h = in.h2;
    if (fused) {
        const LPK_GLOBAL double* __restrict__ pin = to_global(pass == 0 ? in.gpart : in.gpart2);
        for (int j = threadIdx.x; j <= k; j += blockDim.x) {
            double sj = 0.0;
            for (int c = 0; c < in.nseg; ++c) sj += pin[(int64_t)c * in.ldp + j];
            hl[j] = sj;
            if (bx == 0) {
                double* hk = in.H + (int64_t)k * in.ldh;
                if (pass == 0) hk[j] = sj;
                else hk[j] += sj;
            }
        }
        __syncthreads();
        h = hl;
    }
    double acc[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) acc[t] = 0.0;
    chunk_axpy<RPL>(in, in.V, k, w, lane, base, rpl, h, acc);
#pragma unroll
    for (int t = 0; t < RPL; ++t) red[w][lane + 64 * t] = acc[t];
    __syncthreads();
    double q = 0.0;
    if (threadIdx.x < 64 * rpl) {
        const int r = threadIdx.x;
        const int64_t i = base + r;
        double s = 0.0;
        for (int ww = 0; ww < GS_WAVES; ++ww) s += red[ww][r];
        if (i < m) {
            const double un = u[i] - s;
            u[i] = un;
            q = un * un;
        }
    }
    if (pass == 1) {
        // every block reaches this barrier-bearing sum (no early exit above)
        const double r = block_sum(q, sh);
        if (threadIdx.x == 0) in.gpart[bx] = r;
    }
}

#define LPK_SWITCH_RPL(MACRO)         \
    switch (L.gs_rpl) {               \
        case 1: MACRO(1); break;      \
        case 2: MACRO(2); break;      \
        case 4: MACRO(4); break;      \
        default: MACRO(8); break;     \
    }

void b_gs_dots(const BLaunch& L, int pass) {
    hipLaunchKernelGGL(k_gs_dots, dim3(L.gs_dots_grid, L.S), dim3(64 * GS_DOT_WAVES), 0, L.st, L.I, pass);
}

void b_gs_update(const BLaunch& L, int pass) {
    const int fused = L.gs_fused ? 1 : 0;
#define LPK_GU(R) hipLaunchKernelGGL((k_gs_update<R>), dim3(L.gs_nchunks, L.S), dim3(64 * GS_WAVES), 0, L.st, L.I, pass, fused)
    LPK_SWITCH_RPL(LPK_GU)
#undef LPK_GU
}

// h[j] = sum over the segments of the pass's partials (fixed order) into h2; pass 0
// stores column k of H, pass 1 adds to it
__global__ __launch_bounds__(BLOCK) void k_gs_reduce(const Inst* __restrict__ I, int pass) {
    INST;
    if (in.ctl->done) return;
    const int k = in.ctl->k;
    const int j = bx * BLOCK + threadIdx.x;
    if (j > k) return;
    const double* __restrict__ pin = pass == 0 ? in.gpart : in.gpart2;
    double s = 0.0;
    for (int c = 0; c < in.nseg; ++c) s += pin[(int64_t)c * in.ldp + j];
    in.h2[j] = s;
    double* hk = in.H + (int64_t)k * in.ldh;
    if (pass) hk[j] += s;
    else hk[j] = s;
}

void b_gs_reduce(const BLaunch& L, int pass) {
    hipLaunchKernelGGL(k_gs_reduce, dim3(cdiv(L.max_ldp, BLOCK), L.S), dim3(BLOCK), 0, L.st, L.I, pass);
}

// ||u||^2 from the chunk partials, h_{k+1,k} = ||u||, the earlier Givens rotations on
// column k of H, the new rotation, gamma, and the test |gamma_{k+1}| <= tol * beta.
// Rotation i maps (carry_i, h_{i+1}) to the output entry c_i carry_i + s_i h_{i+1} and the
// next carry -s_i carry_i + c_i h_{i+1}: the carries follow the first-order linear
// recurrence carry_{i+1} = a_i carry_i + b_i (a_i = -s_i, b_i = c_i h_{i+1}).  Column k
// and the coefficients are staged through LDS in chunks; inside a chunk each thread
// composes the affine maps of its consecutive entries, a block-wide scan composes the
// threads' maps, and each thread then replays its entries from its starting carry.  The
// depth is log2(BLOCK) barrier steps instead of a chain of length k (|a_i| <= 1, so the
// composed maps stay bounded).
constexpr int GF_CH = 1024;

struct GivensLds {
    double hb[GF_CH], cb[GF_CH], sb[GF_CH], ob[GF_CH];
    double sA[BLOCK / 64], sB[BLOCK / 64];   // the waves' composed maps
    double carry;
};

// Column kc of H (hk, entries 0..kc; h_{kc+1,kc} = hn): the earlier rotations 0..kc-1,
// then the rotation that zeroes hn, and gamma.  Every thread of the block calls it; thread
// 0 gets the return value: false when that rotation degenerates (r = 0), else true with
// *res = |gamma_{kc+1}|.
__device__ bool givens_column(const Inst& in, double* hk, int kc, double hn, GivensLds& g, double* res) {
    if (threadIdx.x == 0) g.carry = hk[0];
    for (int base = 0; base < kc; base += GF_CH) {
        const int len = kc - base < GF_CH ? kc - base : GF_CH;
        __syncthreads();
        for (int t = threadIdx.x; t < len; t += BLOCK) {
            g.hb[t] = hk[base + t + 1];
            g.cb[t] = in.cs[base + t];
            g.sb[t] = in.sn[base + t];
        }
        __syncthreads();
        // this thread's entries [i0, i1) and the composition of their maps, x -> A x + B
        const int per = (len + BLOCK - 1) / BLOCK;
        const int t = threadIdx.x;
        const int i0 = t * per < len ? t * per : len;
        const int i1 = i0 + per < len ? i0 + per : len;
        double A = 1.0, B = 0.0;
        for (int i = i0; i < i1; ++i) {
            const double a = -g.sb[i], b = g.cb[i] * g.hb[i];
            B = a * B + b;
            A = a * A;
        }
        // inclusive scan over the threads: inside each wave by shuffles, then across the
        // waves through LDS; after it, (A, B) composes the maps of threads 0..t
        const int lane = t & 63, w = t >> 6;
        for (int d = 1; d < 64; d <<= 1) {
            const double pa = __shfl_up(A, d, 64), pb = __shfl_up(B, d, 64);
            if (lane >= d) {
                B = A * pb + B;
                A = A * pa;
            }
        }
        if (lane == 63) {
            g.sA[w] = A;
            g.sB[w] = B;
        }
        __syncthreads();
        double PA = 1.0, PB = 0.0;   // the maps of the earlier waves
        for (int q = 0; q < w; ++q) {
            const double a = g.sA[q], b = g.sB[q];
            PB = a * PB + b;
            PA = a * PA;
        }
        B = A * PB + B;
        A = A * PA;
        // starting carry of this thread's entries: the maps of threads 0..t-1 on the carry
        double EA = __shfl_up(A, 1, 64), EB = __shfl_up(B, 1, 64);
        if (lane == 0) {
            EA = PA;
            EB = PB;
        }
        double carry = g.carry;
        if (t > 0) carry = EA * carry + EB;
        for (int i = i0; i < i1; ++i) {
            const double bv = g.hb[i], c = g.cb[i], sv = g.sb[i];
            g.ob[i] = c * carry + sv * bv;
            carry = -sv * carry + c * bv;
        }
        __syncthreads();   // every thread has read the carry
        if (i0 < i1 && i1 == len) g.carry = carry;
        __syncthreads();
        for (int q2 = threadIdx.x; q2 < len; q2 += BLOCK) hk[base + q2] = g.ob[q2];
    }
    __syncthreads();
    if (threadIdx.x != 0) return false;
    const double a = g.carry, b = hn;
    const double r = hypot(a, b);
    if (r == 0.0) return false;
    const double c = a / r, sv = b / r;
    in.cs[kc] = c;
    in.sn[kc] = sv;
    hk[kc] = r;
    hk[kc + 1] = 0.0;
    const double gk = in.gam[kc];
    in.gam[kc + 1] = -sv * gk;
    in.gam[kc] = c * gk;
    *res = fabs(in.gam[kc + 1]);
    return true;
}

// ||u||^2 from the chunk partials, h_{k+1,k} = ||u||, the Givens step on column k, and
// the test |gamma_{k+1}| <= tol * beta.  Rotation i maps (carry_i, h_{i+1}) to the output
// entry c_i carry_i + s_i h_{i+1} and the next carry -s_i carry_i + c_i h_{i+1}: the carries
// follow the first-order linear recurrence carry_{i+1} = a_i carry_i + b_i (a_i = -s_i,
// b_i = c_i h_{i+1}).  Column k and the coefficients are staged through LDS in chunks;
// inside a chunk each thread composes the affine maps of its consecutive entries, a
// block-wide scan composes the threads' maps, and each thread then replays its entries from
// its starting carry.  The depth is log2(BLOCK) barrier steps instead of a chain of length
// k (|a_i| <= 1, so the composed maps stay bounded).
__global__ __launch_bounds__(BLOCK) void k_gs_finish(const Inst* __restrict__ I) {
    __shared__ double sh[BLOCK / 64];
    __shared__ GivensLds g;
    INST;
    KrylovCtl* ctl = in.ctl;
    if (ctl->done) return;
    double q = 0.0;
    for (int c = threadIdx.x; c < in.nchunks; c += BLOCK) q += in.gpart[c];
    const double nrm2 = block_sum(q, sh);
    const int k = ctl->k;
    double* hk = in.H + (int64_t)k * in.ldh;
    double res = 0.0;
    const double hn = sqrt(nrm2);   // thread 0's value is the one used
    const bool ok = givens_column(in, hk, k, hn, g, &res);
    if (threadIdx.x != 0) return;
    if (!ok) {
        ctl->done = 1;
        ctl->iters = k;
        ctl->failed = ctl->res > ctl->thresh;
        return;
    }
    ctl->res = res;
    ctl->k = k + 1;
    ctl->iters = k + 1;
    ctl->inv_h = hn != 0.0 ? 1.0 / hn : 0.0;
    if (res <= ctl->thresh || hn == 0.0 || k + 1 >= ctl->kmax) {
        ctl->done = 1;
        ctl->failed = res > ctl->thresh;
    }
}

void b_gs_finish(const BLaunch& L) {
    hipLaunchKernelGGL(k_gs_finish, dim3(1, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// ------------------------------------------------------------------------------------
// AB-GMRES orthogonalisation with the second pass delayed by one iteration (classical
// Gram-Schmidt twice, reorganised so that each iteration reads the basis twice instead of
// four times).  Iteration k enters with columns 0..k-1 of V orthonormal and column k
// holding v~_k = u~_{k-1} / eta_k: the previous iteration's vector after one projection,
// scaled by an estimate eta_k of its norm, which is what the preconditioner was applied to
// (flexible form: p_k = C v~_k, u_k = A_hat A_hat^T p_k).  Then:
//  * dots: a_j = v_j . v~_k and b_j = v_j . u_k for j < k, c = v~_k . v~_k, d = v~_k . u_k,
//    e = u_k . u_k, all in one pass over V (k_dgs_dots; segment partials as in k_gs_dots);
//  * finish (one block per instance): the second pass of v~_k, t = (a_j), nu^2 = c - ||t||^2,
//    v_k = (v~_k - V t) / nu; so u_{k-1} = V (s' + eta_k t) + eta_k nu v_k, which completes
//    column k-1 of H (s' its first-pass entries), and its Givens step gives the residual
//    after k iterations and the stopping test.  Then u_k's first pass against v_0..v_k:
//    s_j = b_j (j < k), s_k = (d - t . b) / nu, stored as column k of H, and
//    eta_{k+1}^2 = e - ||s||^2 for the next iteration's scaling;
//  * update: v_k = (v~_k - V t) / nu and u~_k = u_k - V s - s_k v_k in one pass over V.
// For k = 0, v_0 = f_hat / beta is exact: no second pass, nu = 1.  Each iteration ends one
// column behind classical Gram-Schmidt twice: the test after k iterations runs in iteration
// k, so a solve runs one more preconditioner application and product than it reports.
// Column k of H needs k < kmax; at k = kmax the iteration only completes column kmax - 1.
// one DPP lane move inside each row of 16 lanes (ctrl: a quad_perm or row-mirror code)
template <int CTRL>
__device__ __forceinline__ double dpp_row_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// The sums over the 64 lanes of eight values at once, each lane keeping half of its values
// at each of the first three levels: lanes 32 apart by permlane32_swap, 16 apart by
// permlane16_swap (gfx950), 8 apart by a row rotation; then xor 1 and xor 2 inside quads and
// the half-row mirror (whose partner then holds the xor-4 partner's sum).  Afterwards the
// eight lanes 8q..8q+7 all hold the sum of v[q].
__device__ __forceinline__ double wave_sum8(const double (&v)[8]) {
    double w[4], x[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v[i]), __double2loint(v[i + 4]), false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v[i]), __double2hiint(v[i + 4]), false, false);
        w[i] = __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(w[i]), __double2loint(w[i + 2]), false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(w[i]), __double2hiint(w[i + 2]), false, false);
        x[i] = __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
    }
    const bool b3 = (threadIdx.x & 8) != 0;
    double y = (b3 ? x[1] : x[0]) + dpp_row_move<0x128>(b3 ? x[0] : x[1]);   // row_ror:8
    y += dpp_row_move<0xB1>(y);
    y += dpp_row_move<0x4E>(y);
    y += dpp_row_move<0x141>(y);
    return y;
}

// The sum over the 64 lanes of one value by the same tree as each of wave_sum8's eight:
// lanes 32 apart, then 16, then 8 (a row rotation), then xor 1, xor 2 and the half-row
// mirror.  Every lane gets the sum; a column's dot is then the same bits whether its task
// reduced one, two or four columns (the column count per task follows the launch width).
__device__ __forceinline__ double wave_sum_tree(double v) {
    {
        const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
        v = __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
    }
    {
        const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
        v = __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
    }
    v = v + dpp_row_move<0x128>(v);   // row_ror:8
    v += dpp_row_move<0xB1>(v);
    v += dpp_row_move<0x4E>(v);
    v += dpp_row_move<0x141>(v);
    return v;
}

// A task is C consecutive columns of one segment: u and v~_k are loaded once per row for
// all of them.  Column k + 1 stands for u itself (its dot with u is u . u).  C = 4 when the
// launch has at least 16384 columns over its instances (the serving mix's long bases), 2 from
// 8192, else 1 (short bases: more, shorter tasks keep more loads in flight).
template <int C>
__device__ __forceinline__ void dgs_dots_tasks(const Inst& in, int k, int blk) {
    const int nseg = in.nseg;
    const int64_t m = in.m;
    const int ngrp = (k + 2 + C - 1) / C;   // columns 0..k, then u . u
    const int tasks = nseg * ngrp;
    const int lane = threadIdx.x & 63;
    const int nw = (int)gridDim.x * GS_DOT_WAVES;
    const LPK_GLOBAL double* __restrict__ u = to_global(in.vec[V_U]);
    const LPK_GLOBAL double* __restrict__ vk = to_global(in.V + (int64_t)k * in.ldv);
    for (int t = blk * GS_DOT_WAVES + (threadIdx.x >> 6); t < tasks; t += nw) {
        const int q = nseg == 1 ? t : t / nseg;
        const int sg = t - q * nseg;
        const int c0 = q * C;
        const int64_t r0 = (int64_t)sg * GS_SEG;
        const int64_t r1 = r0 + GS_SEG < m ? r0 + GS_SEG : m;
        const LPK_GLOBAL double* __restrict__ x[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j = c0 + c;
            x[c] = j <= k ? to_global(in.V + (int64_t)j * in.ldv) : u;   // past k + 1: unused
        }
        const int nc = k + 2 - c0 < C ? k + 2 - c0 : C;
        double a[C], b[C];
#pragma unroll
        for (int c = 0; c < C; ++c) a[c] = b[c] = 0.0;
        constexpr int UNR = C == 1 ? 2 : 1;   // rows in flight per lane
#pragma unroll UNR
        for (int64_t i = r0 + lane; i < r1; i += 64) {
            const double ui = u[i], wi = vk[i];
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (c < nc) {
                    const double xi = x[c][i];
                    a[c] += xi * wi;
                    b[c] += xi * ui;
                }
        }
        if constexpr (C == 4) {
            // the task's eight sums in one pass: lane 8q holds a[q] (q < 4) or b[q - 4]
            const double vv[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
            const double y = wave_sum8(vv);
            const int q = lane >> 3, c = q & 3, j = c0 + c;
            if ((lane & 7) == 0 && c < nc) {
                if (q < 4) {
                    if (j <= k) in.gpart[(int64_t)sg * in.ldp + j] = y;
                } else if (j <= k) {
                    in.gpart2[(int64_t)sg * in.ldp + j] = y;
                } else {
                    in.gpart[(int64_t)sg * in.ldp + j] = y;   // u . u
                }
            }
            continue;
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (c >= nc) break;
            const int j = c0 + c;
            const double sb = wave_sum_tree(b[c]);
            if (j <= k) {
                const double sa = wave_sum_tree(a[c]);
                if (lane == 0) {
                    in.gpart[(int64_t)sg * in.ldp + j] = sa;
                    in.gpart2[(int64_t)sg * in.ldp + j] = sb;
                }
            } else if (lane == 0) {
                in.gpart[(int64_t)sg * in.ldp + j] = sb;   // u . u
            }
        }
    }
}

__global__ __launch_bounds__(64 * GS_DOT_WAVES) void k_dgs_dots(const Inst* __restrict__ I) {
    INST;
    if (in.ctl->done) return;
    const int k = in.ctl->k;
    const int64_t work = (int64_t)(k + 2) * gridDim.y;
    if (work >= 16384) dgs_dots_tasks<4>(in, k, bx);
    else if (work >= 8192) dgs_dots_tasks<2>(in, k, bx);
    else dgs_dots_tasks<1>(in, k, bx);
}

void b_dgs_dots(const BLaunch& L) {
    hipLaunchKernelGGL(k_dgs_dots, dim3(L.gs_dots_grid, L.S), dim3(64 * GS_DOT_WAVES), 0, L.st, L.I);
}

__global__ __launch_bounds__(BLOCK) void k_dgs_finish(const Inst* __restrict__ I) {
    __shared__ double sh3[BLOCK / 64][3];
    __shared__ GivensLds g;
    __shared__ double sc[4];
    INST;
    KrylovCtl* ctl = in.ctl;
    if (ctl->done) return;
    const int k = ctl->k;
    const int nseg = in.nseg;
    double* __restrict__ ta = in.gpart;    // row 0: a_j (j <= k), then e at k + 1
    double* __restrict__ tb = in.gpart2;   // row 0: b_j (j <= k)
    // the segment sums, in place in row 0, in a fixed order
    if (nseg > 1)
        for (int j = threadIdx.x; j <= k + 1; j += BLOCK) {
            double sa = 0.0, sb = 0.0;
            for (int c = 0; c < nseg; ++c) {
                sa += ta[(int64_t)c * in.ldp + j];
                if (j <= k) sb += tb[(int64_t)c * in.ldp + j];
            }
            ta[j] = sa;
            if (j <= k) tb[j] = sb;
        }
    __syncthreads();
    // ||t||^2, t . b and sum_{j<k} b_j^2
    double q1 = 0.0, q2 = 0.0, q3 = 0.0;
    for (int j = threadIdx.x; j < k; j += BLOCK) {
        const double a = ta[j], b = tb[j];
        q1 += a * a;
        q2 += a * b;
        q3 += b * b;
    }
    // the three block sums together (each the same butterfly and wave order as block_sum)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double x1 = __shfl_xor(q1, o, 64), x2 = __shfl_xor(q2, o, 64), x3 = __shfl_xor(q3, o, 64);
        q1 += x1;
        q2 += x2;
        q3 += x3;
    }
    if ((threadIdx.x & 63) == 0) {
        sh3[threadIdx.x >> 6][0] = q1;
        sh3[threadIdx.x >> 6][1] = q2;
        sh3[threadIdx.x >> 6][2] = q3;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        q1 = q2 = q3 = 0.0;
        for (int i = 0; i < BLOCK / 64; ++i) {
            q1 += sh3[i][0];
            q2 += sh3[i][1];
            q3 += sh3[i][2];
        }
        const double c = ta[k], d = tb[k];
        double nu = 1.0, sk = d;
        if (k > 0) {
            const double nu2 = c - q1;
            nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
            sk = nu > 0.0 ? (d - q2) / nu : 0.0;
        }
        sc[0] = nu;
        sc[1] = sk;
        sc[2] = q3 + sk * sk;   // ||s||^2
        sc[3] = ta[k + 1];      // e
    }
    __syncthreads();
    const double nu = sc[0], sk = sc[1];
    if (k > 0) {
        // column k-1: s' (stored there last iteration) + eta_k t, h_{k,k-1} = eta_k nu
        const double eta = ctl->dg_eta;
        double* hc = in.H + (int64_t)(k - 1) * in.ldh;
        for (int j = threadIdx.x; j < k; j += BLOCK) hc[j] += eta * ta[j];
        __syncthreads();
        double res = 0.0;
        const double hn = eta * nu;
        const bool ok = givens_column(in, hc, k - 1, hn, g, &res);
        if (threadIdx.x == 0) {
            if (!ok) {
                ctl->done = 1;
                ctl->iters = k - 1;
                ctl->failed = ctl->res > ctl->thresh;
            } else {
                ctl->res = res;
                ctl->iters = k;
                if (res <= ctl->thresh || hn == 0.0 || k >= ctl->kmax) {
                    ctl->done = 1;
                    ctl->failed = res > ctl->thresh;
                }
            }
            sc[0] = ctl->done;
        }
        __syncthreads();
        if (sc[0] != 0.0) return;
    }
    // u_k's first pass: column k of H, the next scaling, and the update's coefficients
    double* hk = in.H + (int64_t)k * in.ldh;
    for (int j = threadIdx.x; j < k; j += BLOCK) hk[j] = tb[j];
    if (threadIdx.x == 0) {
        hk[k] = sk;
        const double e = sc[3];
        double eta2 = e - sc[2];
        if (eta2 < 1e-24 * e) eta2 = 1e-24 * e;   // cancellation: the next pass rescales
        const double eta = sqrt(eta2);
        ctl->dg_eta = eta;
        ctl->dg_nu = nu;
        ctl->dg_sk = sk;
        ctl->inv_h = eta > 0.0 ? 1.0 / eta : 0.0;
        ctl->k = k + 1;
    }
}

void b_dgs_finish(const BLaunch& L) {
    hipLaunchKernelGGL(k_dgs_finish, dim3(1, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// acc_t[r] += sum_j V[i_r, j] t_j and acc_s[r] += sum_j V[i_r, j] s_j over the wave's
// columns j (w, w + GS_WAVES, ... < kk, increasing), one load of V for both (half the
// single-vector unroll: two accumulators per row; the full unroll measured slower)
template <int RPL>
__device__ __forceinline__ void chunk_axpy2(const Inst& in, int kk, int w, int lane, int64_t base, int rpl,
                                            const double* tc, const double* scf, double (&at)[RPL],
                                            double (&as)[RPL]) {
    constexpr int U = gs_unroll<RPL>() >= 2 ? gs_unroll<RPL>() / 2 : 1;
    const int64_t m = in.m;
    int j = w;
    for (; j + (U - 1) * GS_WAVES < kk; j += U * GS_WAVES) {
        double v[U][RPL], tq[U], sq[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            tq[q] = tc[j + q * GS_WAVES];
            sq[q] = scf[j + q * GS_WAVES];
            const LPK_GLOBAL double* __restrict__ vj = to_global(in.V + (int64_t)(j + q * GS_WAVES) * in.ldv);
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
                const int64_t i = base + lane + 64 * t;
                v[q][t] = (t < rpl && i < m) ? vj[i] : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
                at[t] += v[q][t] * tq[q];
                as[t] += v[q][t] * sq[q];
            }
    }
    for (; j < kk; j += GS_WAVES) {
        const double tj = tc[j], sj = scf[j];
        const LPK_GLOBAL double* __restrict__ vj = to_global(in.V + (int64_t)j * in.ldv);
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int64_t i = base + lane + 64 * t;
            const double x = (t < rpl && i < m) ? vj[i] : 0.0;
            at[t] += x * tj;
            as[t] += x * sj;
        }
    }
}

template <int RPL>
__global__ __launch_bounds__(64 * GS_WAVES) void k_dgs_update(const Inst* __restrict__ I) {
    // the waves' partial sums of both vectors in one pass through LDS when they fit in
    // 16 KiB (RPL <= 2), else one vector after the other through the same LDS
    constexpr bool ONE = RPL <= 2;
    __shared__ double red[ONE ? 2 : 1][GS_WAVES][64 * RPL];
    __shared__ double tl[GS_HLDS / 2], sl[GS_HLDS / 2];
    INST;
    const KrylovCtl* ctl = in.ctl;
    if (ctl->done || bx >= in.nchunks) return;
    const int kk = ctl->k - 1;   // the iteration whose finish ran
    const int rpl = in.rpl;
    const int64_t m = in.m;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)bx * 64 * rpl;
    const double* tc = in.gpart;
    const double* scf = in.gpart2;
    if (kk <= GS_HLDS / 2) {
        for (int j = threadIdx.x; j < kk; j += blockDim.x) {
            tl[j] = tc[j];
            sl[j] = scf[j];
        }
        __syncthreads();
        tc = tl;
        scf = sl;
    }
    double at[RPL], as[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) at[t] = as[t] = 0.0;
    chunk_axpy2<RPL>(in, kk, w, lane, base, rpl, tc, scf, at, as);
    const int r = threadIdx.x;
    double st = 0.0, ss = 0.0;
    if constexpr (ONE) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            red[0][w][lane + 64 * t] = at[t];
            red[ONE ? 1 : 0][w][lane + 64 * t] = as[t];
        }
        __syncthreads();
        if (r < 64 * rpl)
            for (int ww = 0; ww < GS_WAVES; ++ww) {
                st += red[0][ww][r];
                ss += red[ONE ? 1 : 0][ww][r];
            }
    } else {
#pragma unroll
        for (int t = 0; t < RPL; ++t) red[0][w][lane + 64 * t] = at[t];
        __syncthreads();
        if (r < 64 * rpl)
            for (int ww = 0; ww < GS_WAVES; ++ww) st += red[0][ww][r];
        __syncthreads();
#pragma unroll
        for (int t = 0; t < RPL; ++t) red[0][w][lane + 64 * t] = as[t];
        __syncthreads();
        if (r < 64 * rpl)
            for (int ww = 0; ww < GS_WAVES; ++ww) ss += red[0][ww][r];
    }
    if (r < 64 * rpl) {
        const int64_t i = base + r;
        if (i < m) {
            LPK_GLOBAL double* __restrict__ vk = to_global(in.V + (int64_t)kk * in.ldv);
            LPK_GLOBAL double* __restrict__ u = to_global(in.vec[V_U]);
            const double v = (vk[i] - st) / ctl->dg_nu;
            vk[i] = v;
            u[i] = u[i] - ss - v * ctl->dg_sk;
        }
    }
}

void b_dgs_update(const BLaunch& L) {
#define LPK_GU(R) hipLaunchKernelGGL((k_dgs_update<R>), dim3(L.gs_nchunks, L.S), dim3(64 * GS_WAVES), 0, L.st, L.I)
    LPK_SWITCH_RPL(LPK_GU)
#undef LPK_GU
}

// ------------------------------------------------------------------------------------
// solve set-up and solution assembly
__global__ __launch_bounds__(BLOCK) void k_init_rhs(const Inst* __restrict__ I, int pmask) {
    __shared__ double sh[BLOCK / 64];
    INST;
    if (!takes_part(in, pmask) || bx >= in.nbr) return;
    const double* __restrict__ f = in.vec[V_F];
    const double* __restrict__ rho = in.vec[V_RHO];
    double* __restrict__ fh = in.vec[V_FH];
    double* __restrict__ U = in.vec[V_U];
    double q = 0.0;
    const int64_t stride = (int64_t)in.nbr * BLOCK;
    for (int64_t i = (int64_t)bx * BLOCK + threadIdx.x; i < in.m; i += stride) {
        const double v = f[i] / rho[i];
        fh[i] = v;
        U[i] = v;
        q += v * v;
    }
    const double r = block_sum(q, sh);
    write_part(in, bx, 0, r);
}

void b_init_rhs(const BLaunch& L, int pmask) {
    hipLaunchKernelGGL(k_init_rhs, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I, pmask);
}

__global__ __launch_bounds__(BLOCK) void k_init_ctl(const Inst* __restrict__ I, int pmask, int64_t kcap) {
    __shared__ double sh[BLOCK / 64];
    INST;
    KrylovCtl* ctl = in.ctl;
    if (!takes_part(in, pmask)) return;   // other instances keep their solves
    double q = 0.0;
    for (int c = threadIdx.x; c < in.nbr; c += BLOCK) q += in.part[c];
    const double s = block_sum(q, sh);
    if (threadIdx.x != 0) return;
    ctl->k = 0;
    ctl->iters = 0;
    ctl->failed = 0;
    const double beta = sqrt(s);
    int64_t km = in.kmax;
    if (kcap > 0 && kcap < km) km = kcap;
    ctl->active = 1;
    ctl->kmax = (int32_t)km;
    ctl->beta = beta;
    ctl->thresh = in.scal[SC_TOL] * beta;
    ctl->res = beta;
    ctl->res_true = beta;
    ctl->inv_h = beta > 0.0 ? 1.0 / beta : 0.0;
    ctl->omega_c = in.scal[SC_OMC];
    ctl->done = (beta == 0.0 || km <= 0) ? 1 : 0;
    in.gam[0] = beta;
}

void b_init_ctl(const BLaunch& L, int pmask, int64_t kcap) {
    hipLaunchKernelGGL(k_init_ctl, dim3(1, L.S), dim3(BLOCK), 0, L.st, L.I, pmask, kcap);
}

// R y = gamma(1:iters), R the upper triangle of the rotated Hessenberg matrix, by
// columns from the last: y_i = g_i / R_ii, then g_t -= R_ti y_i for t < i.  Up to BS_REG
// iterations, the block stages panels of up to BS_PANEL doubles of H (the columns [c0, c1),
// rows up to c1) into LDS with all its threads, loads in flight together; then wave 0
// applies the panel's columns, lane l holding g_t for t = l + 64 r in registers.  The
// columns of one block of 64 (i >> 6 = RI) run in a loop compiled for RI: y_i's owner is
// register RI, read by every lane with readlane, and only registers r <= RI (rows t < 64
// (RI + 1)) are updated; the others hold rows past i, which the step leaves alone.  Longer
// solves take the same steps with g in memory.  Every entry sees the same operations in
// the same order either way.
constexpr int BS_NR = 16;
constexpr int BS_REG = 64 * BS_NR;
constexpr int BS_PANEL = 18432;   // 144 KiB of LDS (gfx950 gives a workgroup 160 KiB)

__device__ __forceinline__ double readlane_f64(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// columns i = ihi down to ilo (all in the block RI) of the panel starting at column c0 with
// column stride c1
template <int RI>
__device__ __forceinline__ void bs_columns(double (&g)[BS_NR], const double* panel, int c0, int c1, int ihi, int ilo,
                                           int lane) {
    for (int i = ihi; i >= ilo; --i) {
        const double* col = panel + (i - c0) * c1;
        const double yi = readlane_f64(g[RI], i & 63) / col[i];
        // every lane of a register loads (rows t >= i read the diagonal, unused) and selects
        double cv[RI + 1];
#pragma unroll
        for (int r = 0; r <= RI; ++r) {
            const int t = lane + 64 * r;
            cv[r] = col[t < i ? t : i];
        }
#pragma unroll
        for (int r = 0; r <= RI; ++r) {
            const int t = lane + 64 * r;
            const double upd = g[r] - cv[r] * yi;
            g[r] = t == i ? yi : (t < i ? upd : g[r]);
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_backsolve(const Inst* __restrict__ I, int pmask) {
    __shared__ double panel[BS_PANEL];
    INST;
    if (!takes_part(in, pmask)) return;
    const int it = in.ctl->iters;
    double* __restrict__ y = in.ykr;
    if (it > BS_REG) {
        for (int i = threadIdx.x; i < it; i += BLOCK) y[i] = in.gam[i];
        __syncthreads();
        for (int i = it - 1; i >= 0; --i) {
            const double yi = y[i] / in.H[(int64_t)i * in.ldh + i];
            __syncthreads();
            if (threadIdx.x == 0) y[i] = yi;
            for (int t = threadIdx.x; t < i; t += BLOCK) y[t] -= in.H[(int64_t)i * in.ldh + t] * yi;
            __syncthreads();
        }
        return;
    }
    const int lane = threadIdx.x & 63;
    const bool solver = threadIdx.x < 64;
    double g[BS_NR];
#pragma unroll
    for (int r = 0; r < BS_NR; ++r) {
        const int t = lane + 64 * r;
        g[r] = (solver && t < it) ? in.gam[t] : 0.0;
    }
    for (int c1 = it; c1 > 0;) {
        int cb = BS_PANEL / c1;
        if (cb > 64) cb = 64;
        const int c0 = c1 - cb > 0 ? c1 - cb : 0;
        __syncthreads();   // the previous panel is consumed
        // panel[(j - c0) * c1 + t] = H[t, j] for t < c1, j in [c0, c1) (the rows below the
        // diagonal come along unused); eight loads per thread in flight before any store
        const int tot = (c1 - c0) * c1;
        for (int e0 = threadIdx.x; e0 < tot; e0 += 8 * BLOCK) {
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = e0 + q * BLOCK;
                const int j = c0 + e / c1, t = e - (e / c1) * c1;
                v[q] = e < tot ? in.H[(int64_t)j * in.ldh + t] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = e0 + q * BLOCK;
                if (e < tot) panel[e] = v[q];
            }
        }
        __syncthreads();
        if (solver) {
            // the panel's columns by blocks of 64 (at most two blocks: cb <= 64)
            for (int ihi = c1 - 1; ihi >= c0;) {
                const int ri = ihi >> 6;
                const int ilo = std::max(c0, ri * 64);
                switch (ri) {
#define LPK_BS(R_) \
    case R_: bs_columns<R_>(g, panel, c0, c1, ihi, ilo, lane); break;
                    LPK_BS(0) LPK_BS(1) LPK_BS(2) LPK_BS(3) LPK_BS(4) LPK_BS(5) LPK_BS(6) LPK_BS(7)
                    LPK_BS(8) LPK_BS(9) LPK_BS(10) LPK_BS(11) LPK_BS(12) LPK_BS(13) LPK_BS(14) LPK_BS(15)
#undef LPK_BS
                    default: break;
                }
                ihi = ilo - 1;
            }
        }
        c1 = c0;
    }
    if (solver) {
#pragma unroll
        for (int r = 0; r < BS_NR; ++r) {
            const int t = lane + 64 * r;
            if (t < it) y[t] = g[r];
        }
    }
}

void b_backsolve(const BLaunch& L, int pmask) {
    hipLaunchKernelGGL(k_backsolve, dim3(1, L.S), dim3(BLOCK), 0, L.st, L.I, pmask);
}

// dyh = P[:, 0:iters] y  (flexible final step: dw = A_hat^T dyh; BA-GMRES: dyh = V y),
// by row chunks of 64 * RPL rows with the waves of a block splitting the columns, as the
// Gram-Schmidt update
template <int RPL>
__global__ __launch_bounds__(64 * GS_WAVES) void k_combine(const Inst* __restrict__ I, int pmask, int ba) {
    __shared__ double red[GS_WAVES][64 * RPL];
    INST;
    if (!takes_part(in, pmask) || bx >= in.nchunks) return;
    const int it = in.ctl->iters;
    const int rpl = in.rpl;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)bx * 64 * rpl;
    double acc[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) acc[t] = 0.0;
    chunk_axpy<RPL>(in, ba ? in.V : in.P, it - 1, w, lane, base, rpl, in.ykr, acc);
#pragma unroll
    for (int t = 0; t < RPL; ++t) red[w][lane + 64 * t] = acc[t];
    __syncthreads();
    if (threadIdx.x < 64 * rpl) {
        const int64_t i = base + threadIdx.x;
        double s = 0.0;
        for (int ww = 0; ww < GS_WAVES; ++ww) s += red[ww][threadIdx.x];
        if (i < in.m) in.vec[V_DYH][i] = s;
    }
}

void b_combine(const BLaunch& L, int pmask) {
#define LPK_CB(R) \
    hipLaunchKernelGGL((k_combine<R>), dim3(L.gs_nchunks, L.S), dim3(64 * GS_WAVES), 0, L.st, L.I, pmask, L.ba ? 1 : 0)
    LPK_SWITCH_RPL(LPK_CB)
#undef LPK_CB
}

// ------------------------------------------------------------------------------------
// BA-GMRES (eq. ba_ne): GMRES on C A_hat A_hat^T dyh = C f_hat, C the inner-iteration
// operator.  The solve starts once the sweeps have mapped V_U = f_hat to C f_hat:
// partials of ||C f_hat||^2 (nbr blocks, quantity 0), then one block per instance sets
// beta_C = ||C f_hat||, gamma_0 = beta_C, the threshold tol * beta_C (the method's own
// residual, |gamma_k|, is the preconditioned one) and 1 / beta_C, which the next-vector
// kernel applies to form v_0.  ctl->beta stays ||f_hat||, the scale of the true residual.
__global__ __launch_bounds__(BLOCK) void k_ba_norm(const Inst* __restrict__ I, int pmask) {
    __shared__ double sh[BLOCK / 64];
    INST;
    if (!takes_part(in, pmask) || bx >= in.nbr) return;
    const LPK_GLOBAL double* __restrict__ u = to_global(in.vec[V_U]);
    double q = 0.0;
    const int64_t stride = (int64_t)in.nbr * BLOCK;
    for (int64_t i = (int64_t)bx * BLOCK + threadIdx.x; i < in.m; i += stride) q += u[i] * u[i];
    const double r = block_sum(q, sh);
    write_part(in, bx, 0, r);
}

__global__ __launch_bounds__(BLOCK) void k_ba_ctl(const Inst* __restrict__ I, int pmask) {
    __shared__ double sh[BLOCK / 64];
    INST;
    if (!takes_part(in, pmask)) return;
    double q = 0.0;
    for (int c = threadIdx.x; c < in.nbr; c += BLOCK) q += in.part[c];
    const double s = block_sum(q, sh);
    if (threadIdx.x != 0) return;
    KrylovCtl* ctl = in.ctl;
    const double bc = sqrt(s);
    in.gam[0] = bc;
    ctl->res = bc;
    ctl->thresh = in.scal[SC_TOL] * bc;
    ctl->inv_h = bc > 0.0 ? 1.0 / bc : 0.0;
    if (bc == 0.0) ctl->done = 1;
}

void b_ba_start(const BLaunch& L, int pmask) {
    hipLaunchKernelGGL(k_ba_norm, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I, pmask);
    hipLaunchKernelGGL(k_ba_ctl, dim3(1, L.S), dim3(BLOCK), 0, L.st, L.I, pmask);
}

// V[:,k] = u / h_{k,k-1} (u = V_U, 1/h = ctl->inv_h, k = ctl->k) for instances still
// iterating: after the start (k = 0, 1/h = 1/beta_C) and after each Givens step
__global__ __launch_bounds__(BLOCK) void k_ba_vnext(const Inst* __restrict__ I, int pmask) {
    INST;
    const LPK_GLOBAL KrylovCtl* ctl = to_global(in.ctl);
    if (!takes_part(in, pmask) || ctl->done) return;
    const double ih = ctl->inv_h;
    const LPK_GLOBAL double* __restrict__ u = to_global(in.vec[V_U]);
    LPK_GLOBAL double* __restrict__ v = to_global(in.V + (int64_t)ctl->k * in.ldv);
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)bx * BLOCK + threadIdx.x; i < in.m; i += stride) v[i] = u[i] * ih;
}

void b_ba_vnext(const BLaunch& L, int pmask) {
    hipLaunchKernelGGL(k_ba_vnext, dim3(capg(cdiv(L.max_m, BLOCK), GRID_CAP), L.S), dim3(BLOCK), 0, L.st, L.I,
                       pmask);
}

__global__ __launch_bounds__(BLOCK) void k_true_res(const Inst* __restrict__ I, int pmask) {
    __shared__ double sh[BLOCK / 64];
    INST;
    if (!takes_part(in, pmask)) return;
    double q = 0.0;
    for (int c = threadIdx.x; c < in.nbs; c += BLOCK) q += in.part[c];
    const double s = block_sum(q, sh);
    if (threadIdx.x == 0) in.ctl->res_true = sqrt(s);
}

void b_true_res(const BLaunch& L, int pmask) {
    hipLaunchKernelGGL(k_true_res, dim3(1, L.S), dim3(BLOCK), 0, L.st, L.I, pmask);
}

// ------------------------------------------------------------------------------------
// CGNE and MRNE preconditioned by inner iterations (Sec. 3.3), on A_hat dw = f_hat with
// dw_0 = 0.  The preconditioner C is the inner-iteration operator: applied to a vector
// t it gives the multipliers p = C t (column 0 of P) and A_hat^T p (V_Z64, in FP64).
// The multipliers of every n-vector the method forms are carried along, so dyh with
// dw = A_hat^T dyh comes out of the iteration itself.
//
// Vectors.  CGNE: g (residual) = V_U, C g = P0, A_hat^T C g = V_Z64, q = V_Q with its
// multipliers V_QM, A_hat q = V_TMPM.  MRNE: t = A_hat p = V_U, C t = P0,
// v = A_hat^T C t = V_Z64, q = V_Q (multipliers V_QM), p = V_PV (multipliers V_PM); MRNE's
// residual recurrence g is not formed, since nothing reads it here.  Both: the
// least-residual iterate in V_DWB, V_DYB.
//
// Stopping and failure (Sec. 4.2).  After each step the residual f_hat - A_hat dw is
// recomputed by a CSR product (V_TMPM, its squared norm as partials of quantity 0 over
// nbs blocks) and the check tests its norm against tol ||f_hat||.  The check also keeps
// the least residual so far (dw_0 = 0 included): when the new iterate is the least, the
// next step kernel first copies dw and dyh to V_DWB and V_DYB (CG_SAVE); when the solve
// ends above the tolerance with an earlier iterate the least, the assembly copies that one
// back (CG_RESTORE).
//
// Partials (Inst::part, nbr blocks each): CG_DOT the step's numerator or denominator
// dot product, CG_QQ = q.q.  A multi-block kernel reads scalars only from the control
// block (written by earlier launches) and from complete partials; only the one-block
// check kernel writes the control block, so no block reads a scalar that another block
// of the same launch writes.
constexpr int CG_DOT = 1, CG_QQ = 2;

// the sum of the nb partials of quantity q in fixed order, on every thread of the block
__device__ __forceinline__ double part_total(const Inst& in, int q, int nb, double* sh) {
    double v = 0.0;
    for (int c = threadIdx.x; c < nb; c += blockDim.x) v += in.part[q * RED_MAXBLK + c];
    const double r = block_sum(v, sh);
    __syncthreads();
    if (threadIdx.x == 0) sh[0] = r;
    __syncthreads();
    return sh[0];
}

// start: dw = 0, dyh = 0 (also the least-residual copies: dw_0 has residual ||f_hat||),
// q = qm = p = pm = 0; the sweeps read their input unscaled (1/h = 1) from column k = 0
// (MRNE's start: f_hat, written by the start of the solve)
__global__ __launch_bounds__(BLOCK) void k_cg_init(const Inst* __restrict__ I, int pmask, int mrne) {
    INST;
    if (!takes_part(in, pmask)) return;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    const int64_t t0 = (int64_t)bx * BLOCK + threadIdx.x;
    for (int64_t j = t0; j < in.n; j += stride) {
        in.vec[V_DW][j] = 0.0;
        in.vec[V_DWB][j] = 0.0;
        in.vec[V_Q][j] = 0.0;
        in.vec[V_PV][j] = 0.0;
    }
    for (int64_t i = t0; i < in.m; i += stride) {
        in.vec[V_DYH][i] = 0.0;
        in.vec[V_DYB][i] = 0.0;
        in.vec[V_QM][i] = 0.0;
        in.vec[V_PM][i] = 0.0;
    }
    if (bx == 0 && threadIdx.x == 0) {
        KrylovCtl* ctl = in.ctl;
        ctl->k = 0;
        ctl->inv_h = 1.0;
        ctl->cg_gamma = 0.0;
        ctl->cg_beta = 0.0;
        ctl->cg_phase = mrne ? 0 : 1;
        ctl->cg_save = 0;
        ctl->cg_best = ctl->beta;
    }
}

void b_cg_init(const BLaunch& L, int pmask) {
    const unsigned gx = capg(cdiv(L.max_m > L.max_n ? L.max_m : L.max_n, BLOCK), GRID_CAP);
    hipLaunchKernelGGL(k_cg_init, dim3(gx, L.S), dim3(BLOCK), 0, L.st, L.I, pmask, L.krylov == 2 ? 1 : 0);
}

// The loop kernels below run on nbr blocks per instance, each a grid-stride slice of
// the instance's vectors, and return at once for finished instances.
__global__ __launch_bounds__(BLOCK) void k_cg_dot(const Inst* __restrict__ I, int xs, int ys, int nlen) {
    __shared__ double sh[BLOCK / 64];
    INST;
    if (in.ctl->done || bx >= in.nbr || in.ctl->cg_phase == 0) return;
    const double* __restrict__ x = in.vec[xs];
    const double* __restrict__ y = ys == V_PCOL ? in.P : in.vec[ys];
    const int64_t len = nlen ? in.n : in.m;
    const int64_t stride = (int64_t)in.nbr * BLOCK;
    double acc = 0.0;
    for (int64_t i = (int64_t)bx * BLOCK + threadIdx.x; i < len; i += stride) acc += x[i] * y[i];
    write_part(in, bx, CG_DOT, block_sum(acc, sh));
}

void b_cg_dot(const BLaunch& L, int xs, int ys, int nlen) {
    hipLaunchKernelGGL(k_cg_dot, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I, xs, ys, nlen);
}

// CGNE direction: gamma_new = g . C g (the CG_DOT partials), beta = gamma_new / gamma
// (0 for the first direction), q = A_hat^T C g + beta q, qm = C g + beta qm; q.q partials
__global__ __launch_bounds__(BLOCK) void k_cgne_dir(const Inst* __restrict__ I) {
    __shared__ double sh[BLOCK / 64];
    INST;
    if (in.ctl->done || bx >= in.nbr) return;
    const double gnew = part_total(in, CG_DOT, in.nbr, sh);
    const double bk = in.ctl->iters == 0 ? 0.0 : gnew / in.ctl->cg_gamma;
    const int64_t stride = (int64_t)in.nbr * BLOCK, t0 = (int64_t)bx * BLOCK + threadIdx.x;
    const double* __restrict__ uu = in.vec[V_Z64];
    double* __restrict__ q = in.vec[V_Q];
    double qq = 0.0;
    for (int64_t j = t0; j < in.n; j += stride) {
        const double v = uu[j] + bk * q[j];
        q[j] = v;
        qq += v * v;
    }
    const double* __restrict__ zz = in.P;
    double* __restrict__ qm = in.vec[V_QM];
    for (int64_t i = t0; i < in.m; i += stride) qm[i] = zz[i] + bk * qm[i];
    write_part(in, bx, CG_QQ, block_sum(qq, sh));
}

void b_cgne_dir(const BLaunch& L) {
    hipLaunchKernelGGL(k_cgne_dir, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// the step kernels' first task: copy the iterate in dw, dyh to the least-residual
// vectors when the last check found it the least so far
__device__ __forceinline__ void cg_save_best(const Inst& in, int64_t t0, int64_t stride) {
    if (in.ctl->cg_save != CG_SAVE) return;
    const double* __restrict__ dw = in.vec[V_DW];
    double* __restrict__ dwb = in.vec[V_DWB];
    for (int64_t j = t0; j < in.n; j += stride) dwb[j] = dw[j];
    const double* __restrict__ dyh = in.vec[V_DYH];
    double* __restrict__ dyb = in.vec[V_DYB];
    for (int64_t i = t0; i < in.m; i += stride) dyb[i] = dyh[i];
}

// CGNE step: alpha = gamma_new / q.q; dw += alpha q, dyh += alpha qm, g -= alpha A_hat q
// (A_hat q in V_TMPM).  q.q = 0 ends the iteration (in the check).
__global__ __launch_bounds__(BLOCK) void k_cgne_step(const Inst* __restrict__ I) {
    __shared__ double sh[BLOCK / 64];
    INST;
    if (in.ctl->done || bx >= in.nbr) return;
    const int64_t stride = (int64_t)in.nbr * BLOCK, t0 = (int64_t)bx * BLOCK + threadIdx.x;
    cg_save_best(in, t0, stride);
    const double qq = part_total(in, CG_QQ, in.nbr, sh);
    if (qq == 0.0) return;
    const double alpha = part_total(in, CG_DOT, in.nbr, sh) / qq;
    const double* __restrict__ q = in.vec[V_Q];
    double* __restrict__ dw = in.vec[V_DW];
    for (int64_t j = t0; j < in.n; j += stride) dw[j] += alpha * q[j];
    const double* __restrict__ qm = in.vec[V_QM];
    const double* __restrict__ aq = in.vec[V_TMPM];
    double* __restrict__ dyh = in.vec[V_DYH];
    double* __restrict__ g = in.vec[V_U];
    for (int64_t i = t0; i < in.m; i += stride) {
        dyh[i] += alpha * qm[i];
        g[i] -= alpha * aq[i];
    }
}

void b_cgne_step(const BLaunch& L) {
    hipLaunchKernelGGL(k_cgne_step, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// MRNE step.  Start (phase 0): q = A_hat^T C f_hat, qm = C f_hat; q.q partials.  Else,
// with v = A_hat^T C t, t = A_hat p: alpha = gamma / v.p; dw += alpha p, dyh += alpha pm,
// q -= alpha v, qm -= alpha C t; q.q partials.  v.p = 0 ends the iteration (in the check).
__global__ __launch_bounds__(BLOCK) void k_mrne_step(const Inst* __restrict__ I) {
    __shared__ double sh[BLOCK / 64];
    INST;
    if (in.ctl->done || bx >= in.nbr) return;
    const int64_t stride = (int64_t)in.nbr * BLOCK, t0 = (int64_t)bx * BLOCK + threadIdx.x;
    const double* __restrict__ v = in.vec[V_Z64];
    const double* __restrict__ vm = in.P;
    double* __restrict__ q = in.vec[V_Q];
    double* __restrict__ qm = in.vec[V_QM];
    if (in.ctl->cg_phase == 0) {
        double qq = 0.0;
        for (int64_t j = t0; j < in.n; j += stride) {
            q[j] = v[j];
            qq += v[j] * v[j];
        }
        for (int64_t i = t0; i < in.m; i += stride) qm[i] = vm[i];
        write_part(in, bx, CG_QQ, block_sum(qq, sh));
        return;
    }
    cg_save_best(in, t0, stride);
    const double vp = part_total(in, CG_DOT, in.nbr, sh);
    if (vp == 0.0) return;
    const double alpha = in.ctl->cg_gamma / vp;
    const double* __restrict__ pv = in.vec[V_PV];
    double* __restrict__ dw = in.vec[V_DW];
    double qq = 0.0;
    for (int64_t j = t0; j < in.n; j += stride) {
        dw[j] += alpha * pv[j];
        const double w = q[j] - alpha * v[j];
        q[j] = w;
        qq += w * w;
    }
    const double* __restrict__ pm = in.vec[V_PM];
    double* __restrict__ dyh = in.vec[V_DYH];
    for (int64_t i = t0; i < in.m; i += stride) {
        dyh[i] += alpha * pm[i];
        qm[i] -= alpha * vm[i];
    }
    write_part(in, bx, CG_QQ, block_sum(qq, sh));
}

void b_mrne_step(const BLaunch& L) {
    hipLaunchKernelGGL(k_mrne_step, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// One block per instance: the iteration count, res = ||f_hat - A_hat dw|| (from the
// partials of the recomputed residual) and the stopping test res <= tol ||f_hat||, the
// least-residual bookkeeping, or the limit; a zero denominator stops the iteration where
// it is.  CGNE: gamma = g . C g of this step (the next direction's reference).  MRNE:
// start: gamma = q_0 . q_0; after a step: beta = q.q / gamma and gamma = q.q, and
// gamma = 0 stops the iteration.  A solve that ends above the tolerance with an earlier
// iterate of smaller residual is marked CG_RESTORE and reports that residual.
__device__ __forceinline__ void cg_end(KrylovCtl* ctl, double res) {
    ctl->done = 1;
    ctl->failed = res > ctl->thresh;
    if (ctl->failed && ctl->cg_best < res) {
        ctl->cg_save = CG_RESTORE;
        ctl->res = ctl->cg_best;
    } else {
        ctl->cg_save = 0;
        ctl->res = res;
    }
}

__global__ __launch_bounds__(BLOCK) void k_cg_check(const Inst* __restrict__ I, int mrne) {
    __shared__ double sh[BLOCK / 64];
    INST;
    KrylovCtl* ctl = in.ctl;
    if (ctl->done) return;
    const int nb = in.nbr;
    if (mrne && ctl->cg_phase == 0) {
        const double gam = part_total(in, CG_QQ, nb, sh);
        if (threadIdx.x != 0) return;
        ctl->cg_gamma = gam;
        ctl->cg_beta = 0.0;
        ctl->cg_phase = 1;
        if (!(gam > 0.0)) cg_end(ctl, ctl->res);
        return;
    }
    const double den = part_total(in, mrne ? CG_DOT : CG_QQ, nb, sh);
    double r2 = 0.0;
    for (int c = threadIdx.x; c < in.nbs; c += blockDim.x) r2 += in.part[c];
    r2 = block_sum(r2, sh);
    const double other = part_total(in, mrne ? CG_QQ : CG_DOT, nb, sh);
    if (threadIdx.x != 0) return;
    if (den == 0.0) {
        cg_end(ctl, ctl->res);   // no step was taken: the iterate of the last check
        return;
    }
    const double res = sqrt(r2);
    const int it = ctl->iters + 1;
    ctl->iters = it;
    if (!mrne) ctl->cg_gamma = other;
    if (res <= ctl->thresh) {
        cg_end(ctl, res);
        return;
    }
    const bool least = res < ctl->cg_best;
    if (least) ctl->cg_best = res;
    ctl->cg_save = least ? CG_SAVE : 0;
    ctl->res = res;
    if (it >= ctl->kmax) {
        cg_end(ctl, res);
        return;
    }
    if (mrne) {
        ctl->cg_beta = other / ctl->cg_gamma;
        ctl->cg_gamma = other;
        if (!(other > 0.0)) cg_end(ctl, res);
    }
}

void b_cg_check(const BLaunch& L) {
    hipLaunchKernelGGL(k_cg_check, dim3(1, L.S), dim3(BLOCK), 0, L.st, L.I, L.krylov == 2 ? 1 : 0);
}

// MRNE direction: p = q + beta p, pm = qm + beta pm (beta = 0 at the start: p and pm are
// zero then)
__global__ __launch_bounds__(BLOCK) void k_mrne_dir(const Inst* __restrict__ I) {
    INST;
    if (in.ctl->done || bx >= in.nbr) return;
    const double bk = in.ctl->cg_beta;
    const int64_t stride = (int64_t)in.nbr * BLOCK, t0 = (int64_t)bx * BLOCK + threadIdx.x;
    const double* __restrict__ q = in.vec[V_Q];
    double* __restrict__ pv = in.vec[V_PV];
    for (int64_t j = t0; j < in.n; j += stride) pv[j] = q[j] + bk * pv[j];
    const double* __restrict__ qm = in.vec[V_QM];
    double* __restrict__ pm = in.vec[V_PM];
    for (int64_t i = t0; i < in.m; i += stride) pm[i] = qm[i] + bk * pm[i];
}

void b_mrne_dir(const BLaunch& L) {
    hipLaunchKernelGGL(k_mrne_dir, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// assembly of a CGNE / MRNE solve that missed its tolerance: the least-residual iterate
// replaces the last one (Sec. 4.2)
__global__ __launch_bounds__(BLOCK) void k_cg_restore(const Inst* __restrict__ I, int pmask) {
    INST;
    if (!takes_part(in, pmask) || in.ctl->cg_save != CG_RESTORE) return;
    const int64_t stride = (int64_t)gridDim.x * BLOCK, t0 = (int64_t)bx * BLOCK + threadIdx.x;
    const double* __restrict__ dwb = in.vec[V_DWB];
    double* __restrict__ dw = in.vec[V_DW];
    for (int64_t j = t0; j < in.n; j += stride) dw[j] = dwb[j];
    const double* __restrict__ dyb = in.vec[V_DYB];
    double* __restrict__ dyh = in.vec[V_DYH];
    for (int64_t i = t0; i < in.m; i += stride) dyh[i] = dyb[i];
}

void b_cg_restore(const BLaunch& L, int pmask) {
    const unsigned gx = capg(cdiv(L.max_m > L.max_n ? L.max_m : L.max_n, BLOCK), GRID_CAP);
    hipLaunchKernelGGL(k_cg_restore, dim3(gx, L.S), dim3(BLOCK), 0, L.st, L.I, pmask);
}

// ------------------------------------------------------------------------------------
// scaling: d and the predictor's right-hand side input t = d^2 o r_d (MD_RUN); d = 1,
// t = 0 for the starting-point solves (MD_INIT); MD_API keeps the given d
__global__ __launch_bounds__(BLOCK) void k_scaling(const Inst* __restrict__ I) {
    INST;
    const int md = *in.mode;
    if (!(md & MD_SCALE)) return;
    double* __restrict__ d = in.vec[V_D];
    double* __restrict__ t = in.vec[V_TN];
    const double *__restrict__ x = in.vec[V_X], *__restrict__ s = in.vec[V_S], *__restrict__ rd = in.vec[V_RD];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)bx * BLOCK + threadIdx.x; j < in.n; j += stride) {
        if (!(md & MD_INIT)) {
            const double dj = sqrt(x[j] / s[j]);
            d[j] = dj;
            t[j] = dj * dj * rd[j];
        } else {
            d[j] = 1.0;
            t[j] = 0.0;
        }
    }
}

void b_scaling(const BLaunch& L) {
    hipLaunchKernelGGL(k_scaling, dim3(red_blocks(L.max_n), L.S), dim3(BLOCK), 0, L.st, L.I);
}

// rho_i = ||row i of A D||, A_hat row i = (a_ij d_j) / rho_i (Sec. 3.5), FP32 copy in mixed mode
__global__ __launch_bounds__(BLOCK) void k_scale_rows(const Inst* __restrict__ I, int pmask) {
    INST;
    if (!takes_part(in, pmask)) return;
    const int g = in.g_csr;
    const int lane = threadIdx.x & (g - 1);
    const double* __restrict__ d = in.vec[V_D];
    double* __restrict__ rho = in.vec[V_RHO];
    const int64_t total = (int64_t)in.m * g;
    for (int64_t t0 = (int64_t)bx * BLOCK; t0 < total; t0 += (int64_t)gridDim.x * BLOCK) {
        const int64_t tt = t0 + threadIdx.x;
        const int row = (int)(tt / g);
        double q = 0.0;
        int s = 0, e = 0;
        if (row < in.m) {
            s = in.rp[row];
            e = in.rp[row + 1];
            for (int k = s + lane; k < e; k += g) {
                const double v = in.a[k] * d[in.ci[k]];
                q += v * v;
            }
        }
        q = sg_sum(q, g);
        if (row < in.m) {
            const double r = sqrt(q);
            if (lane == 0) rho[row] = r;
            // a sliced row's element k - s sits at slot k - s of its slice
            const int sl0 = in.rsl ? in.rsl[row] : -1;
            for (int k = s + lane; k < e; k += g) {
                const double v = (in.a[k] * d[in.ci[k]]) / r;
                in.ah[k] = v;
                if (in.ah32) in.ah32[k] = (float)v;
                if (sl0 >= 0) {
                    const int q = sl0 + (k - s) * SL_ROWS;
                    in.sl_val[q] = v;
                    if (in.sl_val32) in.sl_val32[q] = (float)v;
                }
            }
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_scale_cols(const Inst* __restrict__ I, int pmask) {
    INST;
    if (!takes_part(in, pmask)) return;
    const double* __restrict__ d = in.vec[V_D];
    const double* __restrict__ rho = in.vec[V_RHO];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)bx * BLOCK + threadIdx.x; j < in.n; j += stride) {
        const double dj = d[j];
        for (int k = in.cp[j]; k < in.cp[j + 1]; ++k) {
            const double v = (in.ac[k] * dj) / rho[in.ri[k]];
            in.ahc[k] = v;
            if (in.ahc32) in.ahc32[k] = (float)v;
        }
    }
}

void b_scale_rows(const BLaunch& L, int pmask) {
    hipLaunchKernelGGL(k_scale_rows, dim3(capg(L.grid_spmv[M_A_CSR], GRID_CAP), L.S), dim3(BLOCK), 0, L.st, L.I, pmask);
}
void b_scale_cols(const BLaunch& L, int pmask) {
    hipLaunchKernelGGL(k_scale_cols, dim3(capg(cdiv(L.max_n, BLOCK), GRID_CAP), L.S), dim3(BLOCK), 0, L.st, L.I, pmask);
}

// one power-iteration step for the Cimmino step 1/lambda: v (V_TMPM) is scaled by
// 1/sqrt(out[0]) from the previous step's norm (first: v = e / sqrt(m))
__global__ __launch_bounds__(BLOCK) void k_power_scale(const Inst* __restrict__ I, int pmask, int first) {
    INST;
    if (!takes_part(in, pmask)) return;
    double* __restrict__ v = in.vec[V_TMPM];
    const double nr = first ? 0.0 : sqrt(in.out[0]);
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)bx * BLOCK + threadIdx.x; i < in.m; i += stride) {
        if (first) v[i] = 1.0 / sqrt((double)in.m);
        else if (nr > 0.0) v[i] = v[i] / nr;
    }
}

void b_power_step(const BLaunch& L, int pmask, int step) {
    // step 0: v = e/sqrt(m); step > 0: v /= ||v|| (norm from the previous step's finish)
    hipLaunchKernelGGL(k_power_scale, dim3(red_blocks(L.max_m), L.S), dim3(BLOCK), 0, L.st, L.I, pmask,
                       step == 0 ? 1 : 0);
    b_spmv(L, M_AH_CSC, V_TMPM, V_TMPN, EPI_PLAIN, -1, -1, pmask, false);
    b_spmv(L, M_AH_CSR, V_TMPN, V_TMPM, EPI_PLAIN, -1, -1, pmask, true);
    const int ops[1] = {0};
    b_red_finish(L, 1, ops, pmask, 1);
}

// omega_c = 1 / lambda, lambda = ||A_hat A_hat^T v|| for the normalised v of the last step
__global__ void k_set_omc(const Inst* __restrict__ I, int pmask) {
    INST;
    if (!takes_part(in, pmask) || threadIdx.x != 0) return;
    const double lam = sqrt(in.out[0]);
    in.scal[SC_OMC] = lam > 0.0 ? 1.0 / lam : 1.0;
}

void b_set_omc(const BLaunch& L, int pmask) {
    hipLaunchKernelGGL(k_set_omc, dim3(1, L.S), dim3(64), 0, L.st, L.I, pmask);
}

// ------------------------------------------------------------------------------------
// reductions: quantity q of a kernel writes part[q * RED_MAXBLK + block]; the finish sums
// (op 0) or takes the minimum (op 1) over the blocks in block order, per instance
struct FinishArgs {
    int nq, which, pmask;
    int ops[RED_NQ];
};

__global__ __launch_bounds__(BLOCK) void k_red_finish(const Inst* __restrict__ I, FinishArgs a) {
    __shared__ double sh[BLOCK / 64];
    INST;
    if (!takes_part(in, a.pmask)) return;
    const int nblk = a.which == 0 ? in.nbr : in.nbs;
    for (int q = 0; q < a.nq; ++q) {
        const double* pq = in.part + (int64_t)q * RED_MAXBLK;
        double v;
        if (a.ops[q] == 1) {
            v = INFINITY;
            for (int c = threadIdx.x; c < nblk; c += BLOCK) v = fmin(v, pq[c]);
            v = block_min(v, sh);
        } else {
            v = 0.0;
            for (int c = threadIdx.x; c < nblk; c += BLOCK) v += pq[c];
            v = block_sum(v, sh);
        }
        if (threadIdx.x == 0) in.out[q] = v;
        __syncthreads();
    }
}

void b_red_finish(const BLaunch& L, int nq, const int* ops, int pmask, int which) {
    FinishArgs a;
    a.nq = nq;
    a.which = which;
    a.pmask = pmask;
    for (int q = 0; q < RED_NQ; ++q) a.ops[q] = q < nq ? ops[q] : 0;
    hipLaunchKernelGGL(k_red_finish, dim3(1, L.S), dim3(BLOCK), 0, L.st, L.I, a);
}

// The interior-point reductions below partition each instance's vectors by its own
// block count nbr (blocks past it return), so every sum is formed in an order that does
// not depend on the other instances of the batch.
#define IPM_PROLOGUE(cond)                                        \
    INST;                                                         \
    if (!(cond) || bx >= in.nbr) return;             \
    const int64_t stride = (int64_t)in.nbr * BLOCK;               \
    const int64_t tid0 = (int64_t)bx * BLOCK + threadIdx.x

// x.s, c.x, ||r_d||^2 over n and b.y, ||r_p||^2 over m
__global__ __launch_bounds__(BLOCK) void k_measures(const Inst* __restrict__ I, int pmask) {
    __shared__ double sh[BLOCK / 64];
    IPM_PROLOGUE(takes_part(in, pmask));
    const double *x = in.vec[V_X], *s = in.vec[V_S], *c = in.vec[V_C], *rd = in.vec[V_RD];
    const double *b = in.vec[V_B], *y = in.vec[V_Y], *rpv = in.vec[V_RP];
    double q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0;
    for (int64_t j = tid0; j < in.n; j += stride) {
        q0 += x[j] * s[j];
        q1 += c[j] * x[j];
        q2 += rd[j] * rd[j];
    }
    for (int64_t i = tid0; i < in.m; i += stride) {
        q3 += b[i] * y[i];
        q4 += rpv[i] * rpv[i];
    }
    double r;
    r = block_sum(q0, sh); write_part(in, bx, 0, r);
    r = block_sum(q1, sh); write_part(in, bx, 1, r);
    r = block_sum(q2, sh); write_part(in, bx, 2, r);
    r = block_sum(q3, sh); write_part(in, bx, 3, r);
    r = block_sum(q4, sh); write_part(in, bx, 4, r);
}

void b_measures(const BLaunch& L, int pmask) {
    hipLaunchKernelGGL(k_measures, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I, pmask);
}

__device__ __forceinline__ double ratio_term(double v, double dv) { return dv < 0.0 ? -v / dv : INFINITY; }

// after the first solve: MD_RUN: dy_af = dyh / rho and the predictor's recovery
// ds = r_d - dw/d, dx = -d^2 ds - x (Sec. 2.2) with the ratio tests; MD_INIT: x = dw
__global__ __launch_bounds__(BLOCK) void k_post1(const Inst* __restrict__ I) {
    __shared__ double sh[BLOCK / 64];
    IPM_PROLOGUE(*in.mode & MD_POST1);
    const int md = *in.mode;
    double mp = INFINITY, mdd = INFINITY;
    const double* __restrict__ dw = in.vec[V_DW];
    if (md & MD_RUN) {
        const double *dyh = in.vec[V_DYH], *rho = in.vec[V_RHO];
        double* dya = in.vec[V_DYA];
        for (int64_t i = tid0; i < in.m; i += stride) dya[i] = dyh[i] / rho[i];
        const double *rd = in.vec[V_RD], *d = in.vec[V_D], *x = in.vec[V_X], *s = in.vec[V_S];
        double *ds = in.vec[V_DSA], *dx = in.vec[V_DXA];
        for (int64_t j = tid0; j < in.n; j += stride) {
            const double dj = d[j];
            const double dsj = rd[j] - dw[j] / dj;
            const double dxj = -dj * dj * dsj - x[j];
            ds[j] = dsj;
            dx[j] = dxj;
            mp = fmin(mp, ratio_term(x[j], dxj));
            mdd = fmin(mdd, ratio_term(s[j], dsj));
        }
    } else {
        double* x = in.vec[V_X];
        for (int64_t j = tid0; j < in.n; j += stride) x[j] = dw[j];
    }
    double r;
    r = block_min(mp, sh); write_part(in, bx, 0, r);
    r = block_min(mdd, sh); write_part(in, bx, 1, r);
}

void b_post1(const BLaunch& L) {
    hipLaunchKernelGGL(k_post1, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// mu_af numerator: sum (x + ap dx)(s + ad ds) for MD_RHS2 instances
__global__ __launch_bounds__(BLOCK) void k_mu_af(const Inst* __restrict__ I) {
    __shared__ double sh[BLOCK / 64];
    IPM_PROLOGUE(*in.mode & MD_MUAF);
    const double ap = in.scal[SC_AP], ad = in.scal[SC_AD];
    const double *x = in.vec[V_X], *s = in.vec[V_S], *dx = in.vec[V_DXA], *ds = in.vec[V_DSA];
    double q = 0.0;
    for (int64_t j = tid0; j < in.n; j += stride) q += (x[j] + ap * dx[j]) * (s[j] + ad * ds[j]);
    const double r = block_sum(q, sh);
    write_part(in, bx, 0, r);
}

void b_mu_af(const BLaunch& L) {
    hipLaunchKernelGGL(k_mu_af, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// input of the second solve's right-hand side f = A t: MD_RHS2: t = (dx_af ds_af - sigma mu)/s
// (the corrector of Sec. 2.2); MD_INIT: t = c (f = A c, for the projection of c)
__global__ __launch_bounds__(BLOCK) void k_rhs2(const Inst* __restrict__ I) {
    IPM_PROLOGUE(*in.mode & MD_RHS2);
    const int md = *in.mode;
    double* __restrict__ t = in.vec[V_TN];
    if (!(md & MD_INIT)) {
        const double smu = in.scal[SC_SMU];
        const double *dxa = in.vec[V_DXA], *dsa = in.vec[V_DSA], *s = in.vec[V_S];
        for (int64_t j = tid0; j < in.n; j += stride) t[j] = (dxa[j] * dsa[j] - smu) / s[j];
    } else {
        const double* c = in.vec[V_C];
        for (int64_t j = tid0; j < in.n; j += stride) t[j] = c[j];
    }
}

void b_rhs2(const BLaunch& L) {
    hipLaunchKernelGGL(k_rhs2, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// after the second solve: MD_RHS2: dy_cc = dyh / rho, dy += dy_cc, the corrector's recovery
// added in place (ds_cc = -dw/d, dx_cc = -d^2 ds_cc - dx_af ds_af / s + sigma mu / s) and
// the ratio tests of the combined direction; MD_INIT: y = dyh / rho, s = c - dw, then
// min x and min s (NaN counts as -inf)
__global__ __launch_bounds__(BLOCK) void k_post2(const Inst* __restrict__ I) {
    __shared__ double sh[BLOCK / 64];
    IPM_PROLOGUE(*in.mode & MD_POST2);
    const int md = *in.mode;
    double q0 = INFINITY, q1 = INFINITY;
    const double *dyh = in.vec[V_DYH], *rho = in.vec[V_RHO], *dw = in.vec[V_DW];
    if (md & MD_INIT) {
        double *y = in.vec[V_Y], *s = in.vec[V_S];
        const double *c = in.vec[V_C], *x = in.vec[V_X];
        for (int64_t i = tid0; i < in.m; i += stride) y[i] = dyh[i] / rho[i];
        for (int64_t j = tid0; j < in.n; j += stride) {
            const double sj = c[j] - dw[j];
            s[j] = sj;
            const double xj = x[j];
            q0 = fmin(q0, isnan(xj) ? -INFINITY : xj);
            q1 = fmin(q1, isnan(sj) ? -INFINITY : sj);
        }
    } else {
        double *dxa = in.vec[V_DXA], *dsa = in.vec[V_DSA];
        const double *x = in.vec[V_X], *s = in.vec[V_S];
        double *dyc = in.vec[V_DYC], *dya = in.vec[V_DYA];
        for (int64_t i = tid0; i < in.m; i += stride) {
            const double v = dyh[i] / rho[i];
            dyc[i] = v;
            dya[i] = dya[i] + v;
        }
        const double smu = in.scal[SC_SMU];
        const double* d = in.vec[V_D];
        for (int64_t j = tid0; j < in.n; j += stride) {
            const double dj = d[j], sj = s[j];
            const double xa = dxa[j], sa = dsa[j];
            const double dsc = -dw[j] / dj;
            const double dxc = -dj * dj * dsc - (xa * sa) / sj + smu / sj;
            const double dxt = xa + dxc, dst = sa + dsc;
            dxa[j] = dxt;
            dsa[j] = dst;
            q0 = fmin(q0, ratio_term(x[j], dxt));
            q1 = fmin(q1, ratio_term(sj, dst));
        }
    }
    double r;
    r = block_min(q0, sh); write_part(in, bx, 0, r);
    r = block_min(q1, sh); write_part(in, bx, 1, r);
}

void b_post2(const BLaunch& L) {
    hipLaunchKernelGGL(k_post2, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// Multiple centrality correctors (Gondzio's multi-corrector method).  The target of a
// corrector: at the trial point (x + tp dx, s + td ds) of the aspiration step lengths, each
// product v is moved into [0.1, 10] sigma mu, r = clip(v) - v with r >= -10 sigma mu; the
// corrector's right-hand side input is t = -r/s (f = A t, a corrector solve as in Sec. 2.2).
constexpr double MCC_BMIN = 0.1, MCC_BMAX = 10.0;

__global__ __launch_bounds__(BLOCK) void k_rhs3(const Inst* __restrict__ I) {
    IPM_PROLOGUE(*in.mode & MD_RHS3);
    const double tp = in.scal[SC_AP], td = in.scal[SC_AD], smu = in.scal[SC_SMU];
    const double lo = MCC_BMIN * smu, hi = MCC_BMAX * smu;
    const double *x = in.vec[V_X], *s = in.vec[V_S], *dx = in.vec[V_DXA], *ds = in.vec[V_DSA];
    double* __restrict__ t = in.vec[V_TN];
    for (int64_t j = tid0; j < in.n; j += stride) {
        const double sj = s[j];
        const double v = (x[j] + tp * dx[j]) * (sj + td * ds[j]);
        const double vt = fmin(fmax(v, lo), hi);
        const double r = fmax(vt - v, -hi);
        t[j] = -r / sj;
    }
}

void b_rhs3(const BLaunch& L) {
    hipLaunchKernelGGL(k_rhs3, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// after a corrector's solve: dyc = dyh / rho, dsc = -dw / d, dxc = -d^2 dsc - t (so that
// S dxc + X dsc = r), kept apart; the ratio minima of (dx + dxc, ds + dsc)
__global__ __launch_bounds__(BLOCK) void k_post3(const Inst* __restrict__ I) {
    __shared__ double sh[BLOCK / 64];
    IPM_PROLOGUE(*in.mode & MD_POST3);
    const double *dyh = in.vec[V_DYH], *rho = in.vec[V_RHO], *dw = in.vec[V_DW], *d = in.vec[V_D];
    const double *x = in.vec[V_X], *s = in.vec[V_S], *dxa = in.vec[V_DXA], *dsa = in.vec[V_DSA];
    const double* t = in.vec[V_TN];
    double *dyc = in.vec[V_DYC], *dxc = in.vec[V_DXC], *dsc = in.vec[V_DSC];
    for (int64_t i = tid0; i < in.m; i += stride) dyc[i] = dyh[i] / rho[i];
    double q0 = INFINITY, q1 = INFINITY;
    for (int64_t j = tid0; j < in.n; j += stride) {
        const double dj = d[j];
        const double sc = -dw[j] / dj;
        const double xc = -dj * dj * sc - t[j];
        dsc[j] = sc;
        dxc[j] = xc;
        q0 = fmin(q0, ratio_term(x[j], dxa[j] + xc));
        q1 = fmin(q1, ratio_term(s[j], dsa[j] + sc));
    }
    double r;
    r = block_min(q0, sh); write_part(in, bx, 0, r);
    r = block_min(q1, sh); write_part(in, bx, 1, r);
}

void b_post3(const BLaunch& L) {
    hipLaunchKernelGGL(k_post3, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// an accepted corrector joins the direction: dx += dxc, ds += dsc, dy += dyc
__global__ __launch_bounds__(BLOCK) void k_mcc_add(const Inst* __restrict__ I) {
    IPM_PROLOGUE(*in.mode & MD_MCCADD);
    double *dxa = in.vec[V_DXA], *dsa = in.vec[V_DSA], *dya = in.vec[V_DYA];
    const double *dxc = in.vec[V_DXC], *dsc = in.vec[V_DSC], *dyc = in.vec[V_DYC];
    for (int64_t j = tid0; j < in.n; j += stride) {
        dxa[j] = dxa[j] + dxc[j];
        dsa[j] = dsa[j] + dsc[j];
    }
    for (int64_t i = tid0; i < in.m; i += stride) dya[i] = dya[i] + dyc[i];
}

void b_mcc_add(const BLaunch& L) {
    hipLaunchKernelGGL(k_mcc_add, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// starting point: x += hx, s += hs; then x.s, sum x, sum s
__global__ __launch_bounds__(BLOCK) void k_shift(const Inst* __restrict__ I, int pmask) {
    __shared__ double sh[BLOCK / 64];
    IPM_PROLOGUE(takes_part(in, pmask));
    const double hx = in.scal[SC_HX], hs = in.scal[SC_HS];
    double *x = in.vec[V_X], *s = in.vec[V_S];
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    for (int64_t j = tid0; j < in.n; j += stride) {
        const double xj = x[j] + hx, sj = s[j] + hs;
        x[j] = xj;
        s[j] = sj;
        q0 += xj * sj;
        q1 += xj;
        q2 += sj;
    }
    double r;
    r = block_sum(q0, sh); write_part(in, bx, 0, r);
    r = block_sum(q1, sh); write_part(in, bx, 1, r);
    r = block_sum(q2, sh); write_part(in, bx, 2, r);
}

void b_shift(const BLaunch& L, int pmask) {
    hipLaunchKernelGGL(k_shift, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I, pmask);
}

// min x and min s (NaN counts as -inf)
__global__ __launch_bounds__(BLOCK) void k_min2(const Inst* __restrict__ I, int pmask) {
    __shared__ double sh[BLOCK / 64];
    IPM_PROLOGUE(takes_part(in, pmask));
    const double *x = in.vec[V_X], *s = in.vec[V_S];
    double a = INFINITY, b = INFINITY;
    for (int64_t j = tid0; j < in.n; j += stride) {
        const double xj = x[j], sj = s[j];
        a = fmin(a, isnan(xj) ? -INFINITY : xj);
        b = fmin(b, isnan(sj) ? -INFINITY : sj);
    }
    double r;
    r = block_min(a, sh); write_part(in, bx, 0, r);
    r = block_min(b, sh); write_part(in, bx, 1, r);
}

void b_min2(const BLaunch& L, int pmask) {
    hipLaunchKernelGGL(k_min2, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I, pmask);
}

// centrality test at the trial point: min_i p_i and sum_i p_i, p_i = (x+ap dx)(s+ad ds),
// into quantities 3 and 4 (0-2 may hold a starting-point phase of other instances)
__global__ __launch_bounds__(BLOCK) void k_backtrack(const Inst* __restrict__ I) {
    __shared__ double sh[BLOCK / 64];
    IPM_PROLOGUE(*in.mode & MD_BT);
    const double ap = in.scal[SC_AP], ad = in.scal[SC_AD];
    const double *x = in.vec[V_X], *s = in.vec[V_S], *dx = in.vec[V_DXA], *ds = in.vec[V_DSA];
    double mn = INFINITY, sm = 0.0;
    for (int64_t j = tid0; j < in.n; j += stride) {
        const double p = (x[j] + ap * dx[j]) * (s[j] + ad * ds[j]);
        mn = fmin(mn, p);
        sm += p;
    }
    double r;
    r = block_min(mn, sh); write_part(in, bx, 3, r);
    r = block_sum(sm, sh); write_part(in, bx, 4, r);
}

void b_backtrack(const BLaunch& L) {
    hipLaunchKernelGGL(k_backtrack, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I);
}

// x += ap dx, s += ad ds, y += ad dy; count entries of x, s that are not finite positive
__global__ __launch_bounds__(BLOCK) void k_update(const Inst* __restrict__ I, int q) {
    __shared__ double sh[BLOCK / 64];
    IPM_PROLOGUE(*in.mode & MD_UPD);
    const double ap = in.scal[SC_AP], ad = in.scal[SC_AD];
    double *x = in.vec[V_X], *s = in.vec[V_S], *y = in.vec[V_Y];
    const double *dx = in.vec[V_DXA], *ds = in.vec[V_DSA], *dy = in.vec[V_DYA];
    double bad = 0.0;
    for (int64_t j = tid0; j < in.n; j += stride) {
        const double xn = x[j] + ap * dx[j];
        const double sn = s[j] + ad * ds[j];
        x[j] = xn;
        s[j] = sn;
        if (!(xn > 0.0) || !(sn > 0.0) || !isfinite(xn) || !isfinite(sn)) bad += 1.0;
    }
    for (int64_t i = tid0; i < in.m; i += stride) y[i] = y[i] + ad * dy[i];
    const double r = block_sum(bad, sh);
    write_part(in, bx, q, r);
}

void b_update(const BLaunch& L, int q) {
    hipLaunchKernelGGL(k_update, dim3(L.max_nbr, L.S), dim3(BLOCK), 0, L.st, L.I, q);
}

// The two parts of a split free variable x = x+ - x- both grow along the central path
// (their dual slacks must both vanish).  After the starting point and after each step, a
// pair whose smaller part exceeds (1 + |x+ - x-|) / 2 is lowered by the excess, both parts
// by the same amount.  Rounded operations throughout (no contraction), so the new parts
// are those of the plain formula.
__global__ __launch_bounds__(BLOCK) void k_free_pairs(const Inst* __restrict__ I, int pmask) {
    INST;
    if (!takes_part(in, pmask) || in.nfpairs == 0) return;
    double* __restrict__ x = in.vec[V_X];
    const int32_t* __restrict__ pr = in.fpairs;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t t = (int64_t)bx * BLOCK + threadIdx.x; t < in.nfpairs; t += stride) {
        const int32_t p = pr[2 * t], q = pr[2 * t + 1];
        const double a = x[p], b = x[q];
        const double lo = a < b ? a : b;
        const double cap = __dmul_rn(0.5, __dadd_rn(1.0, fabs(__dsub_rn(a, b))));
        if (lo > cap) {
            const double d = __dsub_rn(lo, cap);
            x[p] = __dsub_rn(a, d);
            x[q] = __dsub_rn(b, d);
        }
    }
}

void b_free_pairs(const BLaunch& L, int pmask) {
    if (!L.any_free) return;
    hipLaunchKernelGGL(k_free_pairs, dim3(capg(cdiv(L.max_fpairs, BLOCK), GRID_CAP), L.S), dim3(BLOCK), 0, L.st,
                       L.I, pmask);
}

__global__ __launch_bounds__(BLOCK) void k_div_rho(const Inst* __restrict__ I, int dst, int src, int pmask) {
    INST;
    if (!takes_part(in, pmask)) return;
    double* __restrict__ o = in.vec[dst];
    const double *__restrict__ a = in.vec[src], *__restrict__ rho = in.vec[V_RHO];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)bx * BLOCK + threadIdx.x; i < in.m; i += stride) o[i] = a[i] / rho[i];
}

void b_div_rho(const BLaunch& L, int dst, int src, int pmask) {
    hipLaunchKernelGGL(k_div_rho, dim3(red_blocks(L.max_m), L.S), dim3(BLOCK), 0, L.st, L.I, dst, src, pmask);
}

// ------------------------------------------------------------------------------------
// single-instance helpers
__global__ __launch_bounds__(BLOCK) void k_gather(int64_t len, const double* __restrict__ src,
                                                  const int32_t* __restrict__ perm, double* __restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t < len) dst[t] = src[perm[t]];
}
void gather(hipStream_t st, int64_t len, const double* src, const int32_t* perm, double* dst) {
    if (len > 0) hipLaunchKernelGGL(k_gather, dim3(cdiv(len, BLOCK)), dim3(BLOCK), 0, st, len, src, perm, dst);
}
__global__ __launch_bounds__(BLOCK) void k_scatter(int64_t len, const double* __restrict__ src,
                                                   const int32_t* __restrict__ perm, double* __restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t < len) dst[perm[t]] = src[t];
}
void scatter(hipStream_t st, int64_t len, const double* src, const int32_t* perm, double* dst) {
    if (len > 0) hipLaunchKernelGGL(k_scatter, dim3(cdiv(len, BLOCK)), dim3(BLOCK), 0, st, len, src, perm, dst);
}
__global__ __launch_bounds__(BLOCK) void k_fill(int64_t len, double v, double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < len) dst[i] = v;
}
void fill(hipStream_t st, int64_t len, double v, double* dst) {
    if (len > 0) hipLaunchKernelGGL(k_fill, dim3(cdiv(len, BLOCK)), dim3(BLOCK), 0, st, len, v, dst);
}

}  // namespace lpk
