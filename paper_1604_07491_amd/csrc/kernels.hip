// HIP kernels of the interior-point direction path for CDNA4 (gfx950, wave64).
//
// Layout conventions (all device memory):
//  * A is held row-permuted into colour-major order (rows of one colour contiguous) as CSR
//    with int32 row pointers and column indices; the CSC copy indexes the permuted rows.
//  * A_hat = diag(rho)^-1 A D (unit rows, Sec. 3.5) is materialised once per
//    interior-point step in both layouts (FP64) and, for the mixed mode, as FP32 CSR/CSC.
//  * The Krylov basis V and the multiplier vectors P are column-major m x (kmax+1), one
//    contiguous column per basis vector.
// Reductions are two-stage (per-block partials, then one fixed-order pass): results are
// deterministic run to run and no atomics are used.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.h"

namespace lpk {

constexpr int BLOCK = 256;

template <int G, typename T>
__device__ __forceinline__ T sg_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) { return sg_sum<64>(v); }

// block-wide sum, valid on thread 0; sh must hold blockDim.x / 64 doubles
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    return r;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double block_min(double v, double* sh) {
    v = wave_min(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = INFINITY;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = fmin(r, sh[i]);
    return r;
}

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// ------------------------------------------------------------------------------------
// sparse row-dot products (CSR A x; CSC-as-CSR A^T y), one sub-group of G lanes per row
template <int G, typename TV, typename TX, typename TO>
__global__ __launch_bounds__(BLOCK) void k_spmv(int nrows, const int32_t* __restrict__ ptr,
                                                const int32_t* __restrict__ idx,
                                                const TV* __restrict__ val,
                                                const TX* __restrict__ x, TO* __restrict__ out,
                                                int epi, const double* __restrict__ b1,
                                                const double* __restrict__ b2,
                                                const int32_t* __restrict__ skip,
                                                double* __restrict__ part,
                                                const KrylovCtl* __restrict__ xcol,
                                                int64_t xld) {
    __shared__ double sh[BLOCK / 64];
    if (skip && *skip) return;
    if (xcol) x += (int64_t)xcol->k * xld;   // x is column k of a column-major array
    using A = TV;
    const int tid = blockIdx.x * BLOCK + threadIdx.x;
    const int row = tid / G, lane = tid & (G - 1);
    A sum = 0;
    if (row < nrows) {
        const int s = ptr[row], e = ptr[row + 1];
        for (int k = s + lane; k < e; k += G) sum += (A)val[k] * (A)x[idx[k]];
    }
    sum = sg_sum<G>(sum);
    double o = 0.0;
    if (row < nrows && lane == 0) {
        const double sd = (double)sum;
        if (epi == EPI_B_MINUS) o = b1[row] - sd;
        else if (epi == EPI_B1_MINUS_B2) o = b1[row] - sd - b2[row];
        else if (epi == EPI_B_PLUS) o = b1[row] + sd;
        else o = sd;
        out[row] = (TO)o;
    }
    if (part) {
        const double r = block_sum(o * o, sh);
        if (threadIdx.x == 0) part[blockIdx.x] = r;
    }
}

template <typename TV, typename TX, typename TO>
static int launch_spmv(hipStream_t st, int g, int nrows, const int32_t* ptr, const int32_t* idx,
                       const TV* val, const TX* x, TO* out, int epi, const double* b1,
                       const double* b2, const int32_t* skip, double* part,
                       const KrylovCtl* xcol = nullptr, int64_t xld = 0) {
    const unsigned grid = cdiv((int64_t)nrows * g, BLOCK);
    if (grid == 0) return 0;
#define LPK_SPMV(G) hipLaunchKernelGGL((k_spmv<G, TV, TX, TO>), dim3(grid), dim3(BLOCK), 0, st, nrows, ptr, idx, val, x, out, epi, b1, b2, skip, part, xcol, xld)
    switch (g) {
        case 1: LPK_SPMV(1); break;
        case 2: LPK_SPMV(2); break;
        case 4: LPK_SPMV(4); break;
        case 8: LPK_SPMV(8); break;
        case 16: LPK_SPMV(16); break;
        case 32: LPK_SPMV(32); break;
        default: LPK_SPMV(64); break;
    }
#undef LPK_SPMV
    return (int)grid;
}

void spmv_f64(hipStream_t st, int g, int nrows, const int32_t* ptr, const int32_t* idx,
              const double* val, const double* x, double* out, int epi, const double* b1,
              const double* b2, const int32_t* skip) {
    launch_spmv<double, double, double>(st, g, nrows, ptr, idx, val, x, out, epi, b1, b2, skip, nullptr);
}
void spmv_f32(hipStream_t st, int g, int nrows, const int32_t* ptr, const int32_t* idx,
              const float* val, const float* x, float* out, int epi, const double* b1,
              const int32_t* skip) {
    launch_spmv<float, float, float>(st, g, nrows, ptr, idx, val, x, out, epi, b1, nullptr, skip, nullptr);
}
void spmv_f64_col(hipStream_t st, int g, int nrows, const int32_t* ptr, const int32_t* idx,
                  const double* val, const double* X, int64_t ldx, double* out,
                  const KrylovCtl* ctl) {
    launch_spmv<double, double, double>(st, g, nrows, ptr, idx, val, X, out, EPI_PLAIN, nullptr, nullptr,
                                        &ctl->done, nullptr, ctl, ldx);
}
int spmv_f64_nrm(hipStream_t st, int g, int nrows, const int32_t* ptr, const int32_t* idx,
                 const double* val, const double* x, double* out, int epi, const double* b1,
                 double* part) {
    return launch_spmv<double, double, double>(st, g, nrows, ptr, idx, val, x, out, epi, b1, nullptr, nullptr, part);
}

// ------------------------------------------------------------------------------------
// One colour of a NE-SOR sweep (inner iteration of Sec. 3.4 on the unit-row A_hat):
// each row i of the colour, in parallel, computes d = omega (v_i - a_i . z), adds d to
// p_i and d a_i to z.  Rows of one colour share no column, so the z updates are
// disjoint.  The row segment (values, column indices) is held in registers between the
// dot product and the update, so each nonzero is read from memory once per sweep.
template <int G, typename T>
__global__ __launch_bounds__(BLOCK) void k_nesor(int r0, int r1, const int32_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ idx,
                                                 const T* __restrict__ val, T* __restrict__ z,
                                                 const double* __restrict__ V,
                                                 double* __restrict__ P, int64_t ldv,
                                                 double omega, const KrylovCtl* __restrict__ ctl,
                                                 int write_z) {
    if (ctl->done) return;
    const int64_t k = ctl->k;
    const double* __restrict__ v = V + k * ldv;
    double* __restrict__ p = P + k * ldv;
    const int tid = blockIdx.x * BLOCK + threadIdx.x;
    const int row = r0 + tid / G, lane = tid & (G - 1);
    if (row >= r1) return;  // uniform inside the sub-group; no block barrier below
    const int s = ptr[row], e = ptr[row + 1];
    constexpr int R = 8;
    T acc = 0;
    if (e - s <= G * R) {
        T a[R];
        int j[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int kk = s + lane + t * G;
            a[t] = 0;
            j[t] = 0;
            if (kk < e) {
                a[t] = val[kk];
                j[t] = idx[kk];
                acc += a[t] * z[j[t]];
            }
        }
        acc = sg_sum<G>(acc);
        const T delta = (T)omega * ((T)v[row] - acc);
        if (write_z) {
#pragma unroll
            for (int t = 0; t < R; ++t)
                if (s + lane + t * G < e) z[j[t]] += delta * a[t];
        }
        if (lane == 0) p[row] += (double)delta;
    } else {
        for (int kk = s + lane; kk < e; kk += G) acc += val[kk] * z[idx[kk]];
        acc = sg_sum<G>(acc);
        const T delta = (T)omega * ((T)v[row] - acc);
        if (write_z)
            for (int kk = s + lane; kk < e; kk += G) z[idx[kk]] += delta * val[kk];
        if (lane == 0) p[row] += (double)delta;
    }
}

template <typename T>
static void launch_nesor(hipStream_t st, int g, int r0, int r1, const int32_t* ptr,
                         const int32_t* idx, const T* val, T* z, const double* V, double* P,
                         int64_t ldv, double omega, const KrylovCtl* ctl, int write_z) {
    const unsigned grid = cdiv((int64_t)(r1 - r0) * g, BLOCK);
    if (grid == 0) return;
#define LPK_NESOR(G) hipLaunchKernelGGL((k_nesor<G, T>), dim3(grid), dim3(BLOCK), 0, st, r0, r1, ptr, idx, val, z, V, P, ldv, omega, ctl, write_z)
    switch (g) {
        case 1: LPK_NESOR(1); break;
        case 2: LPK_NESOR(2); break;
        case 4: LPK_NESOR(4); break;
        case 8: LPK_NESOR(8); break;
        case 16: LPK_NESOR(16); break;
        case 32: LPK_NESOR(32); break;
        default: LPK_NESOR(64); break;
    }
#undef LPK_NESOR
}

void nesor_colour_f64(hipStream_t st, int g, int r0, int r1, const int32_t* ptr,
                      const int32_t* idx, const double* val, double* z, const double* V,
                      double* P, int64_t ldv, double omega, const KrylovCtl* ctl, int write_z) {
    launch_nesor<double>(st, g, r0, r1, ptr, idx, val, z, V, P, ldv, omega, ctl, write_z);
}
void nesor_colour_f32(hipStream_t st, int g, int r0, int r1, const int32_t* ptr,
                      const int32_t* idx, const float* val, float* z, const double* V,
                      double* P, int64_t ldv, double omega, const KrylovCtl* ctl, int write_z) {
    launch_nesor<float>(st, g, r0, r1, ptr, idx, val, z, V, P, ldv, omega, ctl, write_z);
}

// ------------------------------------------------------------------------------------
// Cimmino inner iterations: r = v - A_hat z (first sweep: z = 0, r = v); p += w r;
// z (+)= w A_hat^T r.
template <int G, typename T>
__global__ __launch_bounds__(BLOCK) void k_cim_res(int m, const int32_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ idx,
                                                   const T* __restrict__ val,
                                                   const T* __restrict__ z,
                                                   const double* __restrict__ V,
                                                   double* __restrict__ P, int64_t ldv,
                                                   double w, T* __restrict__ r, int first,
                                                   const KrylovCtl* __restrict__ ctl) {
    if (ctl->done) return;
    const int64_t k = ctl->k;
    const int tid = blockIdx.x * BLOCK + threadIdx.x;
    const int row = tid / G, lane = tid & (G - 1);
    if (row >= m) return;
    T sum = 0;
    if (!first) {
        const int s = ptr[row], e = ptr[row + 1];
        for (int kk = s + lane; kk < e; kk += G) sum += val[kk] * z[idx[kk]];
        sum = sg_sum<G>(sum);
    }
    if (lane == 0) {
        const T rr = (T)V[k * ldv + row] - sum;
        r[row] = rr;
        P[k * ldv + row] += ctl->omega_c * (double)rr;
    }
}

template <int G, typename T>
__global__ __launch_bounds__(BLOCK) void k_cim_z(int n, const int32_t* __restrict__ cptr,
                                                 const int32_t* __restrict__ ridx,
                                                 const T* __restrict__ cval,
                                                 const T* __restrict__ r, T* __restrict__ z,
                                                 double w, int first,
                                                 const KrylovCtl* __restrict__ ctl) {
    if (ctl->done) return;
    const int tid = blockIdx.x * BLOCK + threadIdx.x;
    const int col = tid / G, lane = tid & (G - 1);
    if (col >= n) return;
    T sum = 0;
    const int s = cptr[col], e = cptr[col + 1];
    for (int kk = s + lane; kk < e; kk += G) sum += cval[kk] * r[ridx[kk]];
    sum = sg_sum<G>(sum);
    const T wc = (T)ctl->omega_c;
    if (lane == 0) z[col] = first ? wc * sum : z[col] + wc * sum;
}

#define LPK_SWITCH_G(MACRO)            \
    switch (g) {                       \
        case 1: MACRO(1); break;       \
        case 2: MACRO(2); break;       \
        case 4: MACRO(4); break;       \
        case 8: MACRO(8); break;       \
        case 16: MACRO(16); break;     \
        case 32: MACRO(32); break;     \
        default: MACRO(64); break;     \
    }

template <typename T>
static void launch_cim_res(hipStream_t st, int g, int m, const int32_t* ptr, const int32_t* idx,
                           const T* val, const T* z, const double* V, double* P, int64_t ldv,
                           double w, T* r, int first, const KrylovCtl* ctl) {
    const unsigned grid = cdiv((int64_t)m * g, BLOCK);
#define LPK_CR(G) hipLaunchKernelGGL((k_cim_res<G, T>), dim3(grid), dim3(BLOCK), 0, st, m, ptr, idx, val, z, V, P, ldv, w, r, first, ctl)
    LPK_SWITCH_G(LPK_CR)
#undef LPK_CR
}
template <typename T>
static void launch_cim_z(hipStream_t st, int g, int n, const int32_t* cptr, const int32_t* ridx,
                         const T* cval, const T* r, T* z, double w, int first, const KrylovCtl* ctl) {
    const unsigned grid = cdiv((int64_t)n * g, BLOCK);
#define LPK_CZ(G) hipLaunchKernelGGL((k_cim_z<G, T>), dim3(grid), dim3(BLOCK), 0, st, n, cptr, ridx, cval, r, z, w, first, ctl)
    LPK_SWITCH_G(LPK_CZ)
#undef LPK_CZ
}

void cimmino_residual_f64(hipStream_t st, int g, int m, const int32_t* ptr, const int32_t* idx,
                          const double* val, const double* z, const double* V, double* P,
                          int64_t ldv, double omega_c, double* r, int first, const KrylovCtl* ctl) {
    launch_cim_res<double>(st, g, m, ptr, idx, val, z, V, P, ldv, omega_c, r, first, ctl);
}
void cimmino_residual_f32(hipStream_t st, int g, int m, const int32_t* ptr, const int32_t* idx,
                          const float* val, const float* z, const double* V, double* P,
                          int64_t ldv, double omega_c, float* r, int first, const KrylovCtl* ctl) {
    launch_cim_res<float>(st, g, m, ptr, idx, val, z, V, P, ldv, omega_c, r, first, ctl);
}
void cimmino_zupdate_f64(hipStream_t st, int g, int n, const int32_t* cptr, const int32_t* ridx,
                         const double* cval, const double* r, double* z, double omega_c, int first,
                         const KrylovCtl* ctl) {
    launch_cim_z<double>(st, g, n, cptr, ridx, cval, r, z, omega_c, first, ctl);
}
void cimmino_zupdate_f32(hipStream_t st, int g, int n, const int32_t* cptr, const int32_t* ridx,
                         const float* cval, const float* r, float* z, double omega_c, int first,
                         const KrylovCtl* ctl) {
    launch_cim_z<float>(st, g, n, cptr, ridx, cval, r, z, omega_c, first, ctl);
}

// ------------------------------------------------------------------------------------
// Krylov loop bookkeeping
__global__ __launch_bounds__(BLOCK) void k_prep(int64_t m, int64_t n, double* __restrict__ V,
                                                const double* __restrict__ U,
                                                double* __restrict__ P, int64_t ldv,
                                                double* __restrict__ z64, float* __restrict__ z32,
                                                const KrylovCtl* __restrict__ ctl) {
    if (ctl->done) return;
    const int64_t k = ctl->k;
    const double ih = ctl->inv_h;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < m; i += stride) {
        V[k * ldv + i] = U[i] * ih;
        P[k * ldv + i] = 0.0;
    }
    if (z64)
        for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) z64[i] = 0.0;
    if (z32)
        for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) z32[i] = 0.0f;
}

void krylov_prep(hipStream_t st, int64_t m, int64_t n, double* V, const double* U, double* P,
                 int64_t ldv, double* z64, float* z32, const KrylovCtl* ctl) {
    int64_t len = (z64 || z32) ? (m > n ? m : n) : m;
    unsigned grid = cdiv(len, BLOCK);
    if (grid > 2048) grid = 2048;
    hipLaunchKernelGGL(k_prep, dim3(grid), dim3(BLOCK), 0, st, m, n, V, U, P, ldv, z64, z32, ctl);
}

__global__ __launch_bounds__(BLOCK) void k_copy_pcol(int64_t m, const double* __restrict__ P,
                                                     int64_t ldv, double* __restrict__ out,
                                                     const KrylovCtl* __restrict__ ctl) {
    if (ctl->done) return;
    const int64_t k = ctl->k;
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < m) out[i] = P[k * ldv + i];
}
void copy_pcol(hipStream_t st, int64_t m, const double* P, int64_t ldv, double* out,
               const KrylovCtl* ctl) {
    hipLaunchKernelGGL(k_copy_pcol, dim3(cdiv(m, BLOCK)), dim3(BLOCK), 0, st, m, P, ldv, out, ctl);
}

// ------------------------------------------------------------------------------------
// Classical Gram-Schmidt applied twice on the tall-skinny basis V (m x (k+1)).
// A block owns a chunk of 64*RPL rows; its waves split the basis columns.
constexpr int GS_WAVES = 8;

GsPlan gs_plan(int64_t m) {
    GsPlan p;
    int rpl = 1;
    while (rpl < 8 && (int64_t)64 * rpl * 1024 < m) rpl *= 2;
    p.rpl = rpl;
    p.nchunks = (int)cdiv(m, 64 * rpl);
    p.waves = GS_WAVES;
    return p;
}

template <int RPL>
__global__ __launch_bounds__(64 * GS_WAVES) void k_gs_dots(int64_t m, const double* __restrict__ V,
                                                           int64_t ldv, const double* __restrict__ u,
                                                           double* __restrict__ part, int64_t ldp,
                                                           const KrylovCtl* __restrict__ ctl) {
    if (ctl->done) return;
    const int k = ctl->k;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * 64 * RPL;
    double uu[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const int64_t i = base + lane + 64 * t;
        uu[t] = i < m ? u[i] : 0.0;
    }
    for (int j = w; j <= k; j += GS_WAVES) {
        const double* __restrict__ vj = V + (int64_t)j * ldv;
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int64_t i = base + lane + 64 * t;
            if (i < m) acc += vj[i] * uu[t];
        }
        acc = wave_sum(acc);
        if (lane == 0) part[(int64_t)blockIdx.x * ldp + j] = acc;
    }
}

constexpr int GS_HLDS = 2048;   // coefficients staged in LDS by the fused reduction

template <int RPL>
__global__ __launch_bounds__(64 * GS_WAVES) void k_gs_update(int64_t m, const double* __restrict__ V,
                                                             int64_t ldv, double* __restrict__ u,
                                                             const double* __restrict__ h,
                                                             double* __restrict__ part, int64_t ldp,
                                                             int mode,
                                                             const KrylovCtl* __restrict__ ctl,
                                                             const double* __restrict__ pin,
                                                             int nchunks, double* __restrict__ H,
                                                             int64_t ldh) {
    __shared__ double red[GS_WAVES][64 * RPL];
    __shared__ double unew[64 * RPL];
    __shared__ double sh[GS_WAVES];
    __shared__ double hl[GS_HLDS];
    if (ctl->done) return;
    const int k = ctl->k;
    if (pin) {
        // fused reduction of the previous pass's dot partials (every block, fixed order);
        // mode 0 follows pass 1 (column k of H = h), mode 1 follows pass 2 (H += h)
        for (int j = threadIdx.x; j <= k; j += blockDim.x) {
            double sj = 0.0;
            for (int c = 0; c < nchunks; ++c) sj += pin[(int64_t)c * ldp + j];
            hl[j] = sj;
            if (blockIdx.x == 0) {
                double* hk = H + (int64_t)k * ldh;
                if (mode == 0) hk[j] = sj;
                else hk[j] += sj;
            }
        }
        __syncthreads();
        h = hl;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * 64 * RPL;
    double acc[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) acc[t] = 0.0;
    for (int j = w; j <= k; j += GS_WAVES) {
        const double hj = h[j];
        const double* __restrict__ vj = V + (int64_t)j * ldv;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int64_t i = base + lane + 64 * t;
            if (i < m) acc[t] += vj[i] * hj;
        }
    }
#pragma unroll
    for (int t = 0; t < RPL; ++t) red[w][lane + 64 * t] = acc[t];
    __syncthreads();
    if (threadIdx.x < 64 * RPL) {
        const int r = threadIdx.x;
        const int64_t i = base + r;
        double s = 0.0;
        for (int ww = 0; ww < GS_WAVES; ++ww) s += red[ww][r];
        double un = 0.0;
        if (i < m) {
            un = u[i] - s;
            u[i] = un;
        }
        unew[r] = un;
    }
    __syncthreads();
    if (mode == 0) {
        double uu[RPL];
#pragma unroll
        for (int t = 0; t < RPL; ++t) uu[t] = unew[lane + 64 * t];
        for (int j = w; j <= k; j += GS_WAVES) {
            const double* __restrict__ vj = V + (int64_t)j * ldv;
            double a = 0.0;
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
                const int64_t i = base + lane + 64 * t;
                if (i < m) a += vj[i] * uu[t];
            }
            a = wave_sum(a);
            if (lane == 0) part[(int64_t)blockIdx.x * ldp + j] = a;
        }
    } else {
        double q = 0.0;
        if (threadIdx.x < 64 * RPL) q = unew[threadIdx.x] * unew[threadIdx.x];
        const double r = block_sum(q, sh);
        if (threadIdx.x == 0) part[blockIdx.x] = r;
    }
}

#define LPK_SWITCH_RPL(MACRO)         \
    switch (pl.rpl) {                 \
        case 1: MACRO(1); break;      \
        case 2: MACRO(2); break;      \
        case 4: MACRO(4); break;      \
        default: MACRO(8); break;     \
    }

void gs_dots(hipStream_t st, const GsPlan& pl, int64_t m, const double* V, int64_t ldv,
             const double* u, double* part, int64_t ldp, const KrylovCtl* ctl) {
#define LPK_GD(R) hipLaunchKernelGGL((k_gs_dots<R>), dim3(pl.nchunks), dim3(64 * GS_WAVES), 0, st, m, V, ldv, u, part, ldp, ctl)
    LPK_SWITCH_RPL(LPK_GD)
#undef LPK_GD
}

void gs_update(hipStream_t st, const GsPlan& pl, int64_t m, const double* V, int64_t ldv,
               double* u, const double* h, double* part, int64_t ldp, int mode,
               const KrylovCtl* ctl) {
    const double* pin = nullptr;
    double* H = nullptr;
    int64_t ldh = 0;
#define LPK_GU(R) hipLaunchKernelGGL((k_gs_update<R>), dim3(pl.nchunks), dim3(64 * GS_WAVES), 0, st, m, V, ldv, u, h, part, ldp, mode, ctl, pin, pl.nchunks, H, ldh)
    LPK_SWITCH_RPL(LPK_GU)
#undef LPK_GU
}

bool gs_fusable(const GsPlan& pl, int64_t kmax) { return pl.nchunks <= 32 && kmax + 1 <= GS_HLDS; }

void gs_update_fused(hipStream_t st, const GsPlan& pl, int64_t m, const double* V, int64_t ldv,
                     double* u, const double* pin, double* part, int64_t ldp, int mode,
                     double* H, int64_t ldh, const KrylovCtl* ctl) {
    const double* h = nullptr;
#define LPK_GUF(R) hipLaunchKernelGGL((k_gs_update<R>), dim3(pl.nchunks), dim3(64 * GS_WAVES), 0, st, m, V, ldv, u, h, part, ldp, mode, ctl, pin, pl.nchunks, H, ldh)
    LPK_SWITCH_RPL(LPK_GUF)
#undef LPK_GUF
}

// h[j] = sum over chunks of part[c, j] (fixed order).  Pass 1 (accumulate == 0) stores
// it in column k of H and in h2; pass 2 stores it in h2 and adds it to column k of H.
__global__ __launch_bounds__(BLOCK) void k_gs_reduce(int nchunks, const double* __restrict__ part,
                                                     int64_t ldp, double* __restrict__ H,
                                                     int64_t ldh, double* __restrict__ h2,
                                                     int accumulate,
                                                     const KrylovCtl* __restrict__ ctl) {
    if (ctl->done) return;
    const int k = ctl->k;
    const int j = blockIdx.x * BLOCK + threadIdx.x;
    if (j > k) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * ldp + j];
    h2[j] = s;
    double* hk = H + (int64_t)k * ldh;
    if (accumulate) hk[j] += s;
    else hk[j] = s;
}

void gs_reduce(hipStream_t st, const GsPlan& pl, const double* part, int64_t ldp, double* H,
               int64_t ldh, double* h2, int accumulate, const KrylovCtl* ctl) {
    hipLaunchKernelGGL(k_gs_reduce, dim3(cdiv(ldp, BLOCK)), dim3(BLOCK), 0, st, pl.nchunks, part,
                       ldp, H, ldh, h2, accumulate, ctl);
}

// ||u||^2 from the chunk partials, h_{k+1,k} = ||u||, the earlier Givens rotations on
// column k of H, the new rotation, gamma, and the stopping test |gamma_{k+1}| <= tol*beta.
__global__ __launch_bounds__(BLOCK) void k_gs_finish(int nchunks, const double* __restrict__ part,
                                                     double* __restrict__ H, int64_t ldh,
                                                     double* __restrict__ cs,
                                                     double* __restrict__ sn,
                                                     double* __restrict__ gam,
                                                     KrylovCtl* __restrict__ ctl) {
    __shared__ double sh[BLOCK / 64];
    if (ctl->done) return;
    double q = 0.0;
    for (int c = threadIdx.x; c < nchunks; c += BLOCK) q += part[c];
    const double nrm2 = block_sum(q, sh);
    if (threadIdx.x != 0) return;
    const int k = ctl->k;
    const double hn = sqrt(nrm2);
    double* hk = H + (int64_t)k * ldh;
    // earlier rotations on column k; the rotated entry i+1 is carried in a register, so
    // the loads of cs, sn and hk do not wait on the previous step
    double carry = hk[0];
#pragma unroll 8
    for (int i = 0; i < k; ++i) {
        const double b = hk[i + 1], c = cs[i], s = sn[i];
        hk[i] = c * carry + s * b;
        carry = -s * carry + c * b;
    }
    const double a = carry, b = hn;
    const double r = hypot(a, b);
    if (r == 0.0) {
        ctl->done = 1;
        ctl->iters = k;
        ctl->failed = ctl->res > ctl->thresh;
        return;
    }
    const double c = a / r, s = b / r;
    cs[k] = c;
    sn[k] = s;
    hk[k] = r;
    hk[k + 1] = 0.0;
    const double g = gam[k];
    gam[k + 1] = -s * g;
    gam[k] = c * g;
    const double res = fabs(gam[k + 1]);
    ctl->res = res;
    ctl->k = k + 1;
    ctl->iters = k + 1;
    ctl->inv_h = hn != 0.0 ? 1.0 / hn : 0.0;
    if (res <= ctl->thresh || hn == 0.0 || k + 1 >= ctl->kmax) {
        ctl->done = 1;
        ctl->failed = res > ctl->thresh;
    }
}

void gs_finish(hipStream_t st, const GsPlan& pl, const double* part, double* H, int64_t ldh,
               double* cs, double* sn, double* gam, KrylovCtl* ctl) {
    hipLaunchKernelGGL(k_gs_finish, dim3(1), dim3(BLOCK), 0, st, pl.nchunks, part, H, ldh, cs, sn,
                       gam, ctl);
}

// ------------------------------------------------------------------------------------
// solve setup and solution assembly
__global__ __launch_bounds__(BLOCK) void k_init_rhs(int64_t m, const double* __restrict__ f,
                                                    const double* __restrict__ rho,
                                                    double* __restrict__ fh,
                                                    double* __restrict__ U,
                                                    double* __restrict__ part) {
    __shared__ double sh[BLOCK / 64];
    double q = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < m; i += stride) {
        const double v = f[i] / rho[i];
        fh[i] = v;
        U[i] = v;
        q += v * v;
    }
    const double r = block_sum(q, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

int red_blocks(int64_t len) {
    int64_t b = (len + BLOCK * 4 - 1) / (BLOCK * 4);
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

void krylov_init_rhs(hipStream_t st, int64_t m, const double* f, const double* rho, double* fh,
                     double* U, double* part, int* nblk_out) {
    // U is the vector the first prep normalises into V[:,0]
    const int nb = red_blocks(m);
    hipLaunchKernelGGL(k_init_rhs, dim3(nb), dim3(BLOCK), 0, st, m, f, rho, fh, U, part);
    *nblk_out = nb;
}

__global__ __launch_bounds__(BLOCK) void k_init_ctl(int nblk, const double* __restrict__ part,
                                                    double tol, int kmax,
                                                    KrylovCtl* __restrict__ ctl,
                                                    double* __restrict__ gam, double omega_c) {
    __shared__ double sh[BLOCK / 64];
    double q = 0.0;
    for (int c = threadIdx.x; c < nblk; c += BLOCK) q += part[c];
    const double s = block_sum(q, sh);
    if (threadIdx.x != 0) return;
    const double beta = sqrt(s);
    ctl->k = 0;
    ctl->iters = 0;
    ctl->failed = 0;
    ctl->kmax = kmax;
    ctl->beta = beta;
    ctl->thresh = tol * beta;
    ctl->res = beta;
    ctl->res_true = beta;
    ctl->inv_h = beta > 0.0 ? 1.0 / beta : 0.0;
    ctl->done = (beta == 0.0 || kmax <= 0) ? 1 : 0;
    ctl->omega_c = omega_c;
    gam[0] = beta;
}

void krylov_init_ctl(hipStream_t st, int64_t m, const double* part, int nblk, const double* fh,
                     double* V, double tol, int kmax, KrylovCtl* ctl, double* gam, double omega_c) {
    (void)m;
    (void)fh;
    (void)V;
    hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(BLOCK), 0, st, nblk, part, tol, kmax, ctl, gam, omega_c);
}

// R y = gamma(1:iters), R = upper triangle of the rotated Hessenberg matrix (column-major)
__global__ __launch_bounds__(BLOCK) void k_backsolve(const double* __restrict__ H, int64_t ldh,
                                                     const double* __restrict__ gam,
                                                     double* __restrict__ y,
                                                     const KrylovCtl* __restrict__ ctl) {
    const int it = ctl->iters;
    for (int i = threadIdx.x; i < it; i += BLOCK) y[i] = gam[i];
    __syncthreads();
    for (int i = it - 1; i >= 0; --i) {
        const double yi = y[i] / H[(int64_t)i * ldh + i];
        __syncthreads();
        if (threadIdx.x == 0) y[i] = yi;
        for (int t = threadIdx.x; t < i; t += BLOCK) y[t] -= H[(int64_t)i * ldh + t] * yi;
        __syncthreads();
    }
}

void krylov_backsolve(hipStream_t st, const double* H, int64_t ldh, const double* gam, double* y,
                      KrylovCtl* ctl) {
    hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(BLOCK), 0, st, H, ldh, gam, y, ctl);
}

// dyh = sum_j P[:, j] y_j  (flexible final step: dw = A_hat^T dyh)
__global__ __launch_bounds__(BLOCK) void k_combine(int64_t m, const double* __restrict__ P,
                                                   int64_t ldv, const double* __restrict__ y,
                                                   double* __restrict__ dyh,
                                                   const KrylovCtl* __restrict__ ctl) {
    const int it = ctl->iters;
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int j = 0; j < it; ++j) s += P[(int64_t)j * ldv + i] * y[j];
    dyh[i] = s;
}

void krylov_combine(hipStream_t st, int64_t m, const double* P, int64_t ldv, const double* y,
                    double* dyh, const KrylovCtl* ctl) {
    hipLaunchKernelGGL(k_combine, dim3(cdiv(m, BLOCK)), dim3(BLOCK), 0, st, m, P, ldv, y, dyh, ctl);
}

__global__ __launch_bounds__(BLOCK) void k_true_res(int nblk, const double* __restrict__ part,
                                                    KrylovCtl* __restrict__ ctl) {
    __shared__ double sh[BLOCK / 64];
    double q = 0.0;
    for (int c = threadIdx.x; c < nblk; c += BLOCK) q += part[c];
    const double s = block_sum(q, sh);
    if (threadIdx.x == 0) ctl->res_true = sqrt(s);
}

void krylov_true_res(hipStream_t st, const double* part, int nblk, KrylovCtl* ctl) {
    hipLaunchKernelGGL(k_true_res, dim3(1), dim3(BLOCK), 0, st, nblk, part, ctl);
}

// ------------------------------------------------------------------------------------
// reductions: quantity q of a kernel writes part[q * maxblk + block]; red_finish reduces
// each quantity over its blocks in block order (op 0 = sum, 1 = min)
struct FinishArgs {
    int nq;
    int nblk;
    int maxblk;
    int ops[8];
};

__global__ __launch_bounds__(BLOCK) void k_red_finish(const double* __restrict__ part,
                                                      double* __restrict__ out, FinishArgs a) {
    __shared__ double sh[BLOCK / 64];
    for (int q = 0; q < a.nq; ++q) {
        const double* pq = part + (int64_t)q * a.maxblk;
        double v;
        if (a.ops[q] == 1) {
            v = INFINITY;
            for (int c = threadIdx.x; c < a.nblk; c += BLOCK) v = fmin(v, pq[c]);
            v = block_min(v, sh);
        } else {
            v = 0.0;
            for (int c = threadIdx.x; c < a.nblk; c += BLOCK) v += pq[c];
            v = block_sum(v, sh);
        }
        if (threadIdx.x == 0) out[q] = v;
        __syncthreads();
    }
}

void red_finish(hipStream_t st, const Red& r, int nq, int nblk, const int* ops) {
    FinishArgs a;
    a.nq = nq;
    a.nblk = nblk;
    a.maxblk = r.maxblk;
    for (int q = 0; q < 8; ++q) a.ops[q] = q < nq ? ops[q] : 0;
    hipLaunchKernelGGL(k_red_finish, dim3(1), dim3(BLOCK), 0, st, r.part, r.out, a);
}

// x.s, c.x, ||rd||^2 over n and b.y, ||rp||^2 over m (one grid covers both ranges)
__global__ __launch_bounds__(BLOCK) void k_measures(int64_t m, int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ s,
                                                    const double* __restrict__ c,
                                                    const double* __restrict__ rd,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ rpv,
                                                    double* __restrict__ part, int maxblk) {
    __shared__ double sh[BLOCK / 64];
    double q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += stride) {
        q0 += x[j] * s[j];
        q1 += c[j] * x[j];
        q2 += rd[j] * rd[j];
    }
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < m; i += stride) {
        q3 += b[i] * y[i];
        q4 += rpv[i] * rpv[i];
    }
    double r;
    r = block_sum(q0, sh); if (threadIdx.x == 0) part[0 * maxblk + blockIdx.x] = r;
    r = block_sum(q1, sh); if (threadIdx.x == 0) part[1 * maxblk + blockIdx.x] = r;
    r = block_sum(q2, sh); if (threadIdx.x == 0) part[2 * maxblk + blockIdx.x] = r;
    r = block_sum(q3, sh); if (threadIdx.x == 0) part[3 * maxblk + blockIdx.x] = r;
    r = block_sum(q4, sh); if (threadIdx.x == 0) part[4 * maxblk + blockIdx.x] = r;
}

void ipm_measures(hipStream_t st, const Red& r, int64_t m, int64_t n, const double* x,
                  const double* s, const double* c, const double* rd, const double* b,
                  const double* y, const double* rpv) {
    const int nb = red_blocks(n > m ? n : m);
    hipLaunchKernelGGL(k_measures, dim3(nb), dim3(BLOCK), 0, st, m, n, x, s, c, rd, b, y, rpv, r.part, r.maxblk);
    const int ops[5] = {0, 0, 0, 0, 0};
    red_finish(st, r, 5, nb, ops);
}

// d = sqrt(x / s), t = d^2 o rd (right-hand side input of the predictor)
__global__ __launch_bounds__(BLOCK) void k_scaling(int64_t n, const double* __restrict__ x,
                                                   const double* __restrict__ s,
                                                   const double* __restrict__ rd,
                                                   double* __restrict__ d, double* __restrict__ t) {
    const int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (j >= n) return;
    const double dj = sqrt(x[j] / s[j]);
    d[j] = dj;
    if (t) t[j] = dj * dj * rd[j];
}

void ipm_scaling(hipStream_t st, int64_t n, const double* x, const double* s, const double* rd,
                 double* d, double* t) {
    hipLaunchKernelGGL(k_scaling, dim3(cdiv(n, BLOCK)), dim3(BLOCK), 0, st, n, x, s, rd, d, t);
}

// rho_i = ||row i of A D||, A_hat row i = (a_ij d_j) / rho_i (Sec. 3.5); FP32 copy too
template <int G>
__global__ __launch_bounds__(BLOCK) void k_scale_rows(int m, const int32_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ idx,
                                                      const double* __restrict__ a,
                                                      const double* __restrict__ d,
                                                      double* __restrict__ rho,
                                                      double* __restrict__ ah,
                                                      float* __restrict__ ah32) {
    const int tid = blockIdx.x * BLOCK + threadIdx.x;
    const int row = tid / G, lane = tid & (G - 1);
    if (row >= m) return;
    const int s = ptr[row], e = ptr[row + 1];
    double q = 0.0;
    for (int k = s + lane; k < e; k += G) {
        const double v = a[k] * (d ? d[idx[k]] : 1.0);
        q += v * v;
    }
    q = sg_sum<G>(q);
    const double r = sqrt(q);
    if (lane == 0) rho[row] = r;
    for (int k = s + lane; k < e; k += G) {
        const double v = (a[k] * (d ? d[idx[k]] : 1.0)) / r;
        ah[k] = v;
        if (ah32) ah32[k] = (float)v;
    }
}

void scale_rows(hipStream_t st, int g, int m, const int32_t* ptr, const int32_t* idx,
                const double* a, const double* d, double* rho, double* ah, float* ah32) {
    const unsigned grid = cdiv((int64_t)m * g, BLOCK);
#define LPK_SR(G) hipLaunchKernelGGL((k_scale_rows<G>), dim3(grid), dim3(BLOCK), 0, st, m, ptr, idx, a, d, rho, ah, ah32)
    LPK_SWITCH_G(LPK_SR)
#undef LPK_SR
}

__global__ __launch_bounds__(BLOCK) void k_scale_cols(int n, const int32_t* __restrict__ cptr,
                                                      const int32_t* __restrict__ ridx,
                                                      const double* __restrict__ ac,
                                                      const double* __restrict__ d,
                                                      const double* __restrict__ rho,
                                                      double* __restrict__ ahc,
                                                      float* __restrict__ ahc32) {
    const int j = blockIdx.x * BLOCK + threadIdx.x;
    if (j >= n) return;
    const double dj = d ? d[j] : 1.0;
    for (int k = cptr[j]; k < cptr[j + 1]; ++k) {
        const double v = (ac[k] * dj) / rho[ridx[k]];
        ahc[k] = v;
        if (ahc32) ahc32[k] = (float)v;
    }
}

void scale_cols(hipStream_t st, int n, const int32_t* cptr, const int32_t* ridx, const double* ac,
                const double* d, const double* rho, double* ahc, float* ahc32) {
    hipLaunchKernelGGL(k_scale_cols, dim3(cdiv(n, BLOCK)), dim3(BLOCK), 0, st, n, cptr, ridx, ac, d, rho, ahc, ahc32);
}

// ratio-test term for one pair: -v/dv where dv < 0, else +inf
__device__ __forceinline__ double ratio_term(double v, double dv) {
    return dv < 0.0 ? -v / dv : INFINITY;
}

// predictor recovery (eq. step_predictor): ds = rd - dw/d, dx = -d^2 ds - x; ratio tests
__global__ __launch_bounds__(BLOCK) void k_recover_af(int64_t n, const double* __restrict__ rd,
                                                      const double* __restrict__ dw,
                                                      const double* __restrict__ d,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ s,
                                                      double* __restrict__ ds,
                                                      double* __restrict__ dx,
                                                      double* __restrict__ part, int maxblk) {
    __shared__ double sh[BLOCK / 64];
    double mp = INFINITY, md = INFINITY;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += stride) {
        const double dj = d[j];
        const double dsj = rd[j] - dw[j] / dj;
        const double dxj = -dj * dj * dsj - x[j];
        ds[j] = dsj;
        dx[j] = dxj;
        mp = fmin(mp, ratio_term(x[j], dxj));
        md = fmin(md, ratio_term(s[j], dsj));
    }
    double r;
    r = block_min(mp, sh); if (threadIdx.x == 0) part[0 * maxblk + blockIdx.x] = r;
    r = block_min(md, sh); if (threadIdx.x == 0) part[1 * maxblk + blockIdx.x] = r;
}

void ipm_recover_af(hipStream_t st, const Red& r, int64_t n, const double* rd, const double* dw,
                    const double* d, const double* x, const double* s, double* ds, double* dx) {
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_recover_af, dim3(nb), dim3(BLOCK), 0, st, n, rd, dw, d, x, s, ds, dx, r.part, r.maxblk);
    const int ops[2] = {1, 1};
    red_finish(st, r, 2, nb, ops);
}

__global__ __launch_bounds__(BLOCK) void k_mu_af(int64_t n, const double* __restrict__ x,
                                                 const double* __restrict__ s,
                                                 const double* __restrict__ dx,
                                                 const double* __restrict__ ds, double ap,
                                                 double ad, double* __restrict__ part) {
    __shared__ double sh[BLOCK / 64];
    double q = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += stride)
        q += (x[j] + ap * dx[j]) * (s[j] + ad * ds[j]);
    const double r = block_sum(q, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

void ipm_mu_af(hipStream_t st, const Red& r, int64_t n, const double* x, const double* s,
               const double* dx, const double* ds, double ap, double ad) {
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_mu_af, dim3(nb), dim3(BLOCK), 0, st, n, x, s, dx, ds, ap, ad, r.part);
    const int ops[1] = {0};
    red_finish(st, r, 1, nb, ops);
}

// corrector right-hand side input: t = (dx_af o ds_af - sigma mu) / s
__global__ __launch_bounds__(BLOCK) void k_cc_rhs(int64_t n, const double* __restrict__ dxa,
                                                  const double* __restrict__ dsa,
                                                  const double* __restrict__ s, double smu,
                                                  double* __restrict__ t) {
    const int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (j < n) t[j] = (dxa[j] * dsa[j] - smu) / s[j];
}

void ipm_cc_rhs(hipStream_t st, int64_t n, const double* dxa, const double* dsa, const double* s,
                double smu, double* t) {
    hipLaunchKernelGGL(k_cc_rhs, dim3(cdiv(n, BLOCK)), dim3(BLOCK), 0, st, n, dxa, dsa, s, smu, t);
}

// corrector recovery (eq. step_corrector) added to the predictor direction in place:
// ds_cc = -dw/d; dx_cc = -d^2 ds_cc - (dx_af ds_af)/s + sigma mu / s; ratio tests
__global__ __launch_bounds__(BLOCK) void k_recover_cc(int64_t n, const double* __restrict__ dw,
                                                      const double* __restrict__ d,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ s, double smu,
                                                      double* __restrict__ dxa,
                                                      double* __restrict__ dsa,
                                                      double* __restrict__ part, int maxblk) {
    __shared__ double sh[BLOCK / 64];
    double mp = INFINITY, md = INFINITY;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += stride) {
        const double dj = d[j], sj = s[j];
        const double xa = dxa[j], sa = dsa[j];
        const double dsc = -dw[j] / dj;
        const double dxc = -dj * dj * dsc - (xa * sa) / sj + smu / sj;
        const double dxt = xa + dxc, dst = sa + dsc;
        dxa[j] = dxt;
        dsa[j] = dst;
        mp = fmin(mp, ratio_term(x[j], dxt));
        md = fmin(md, ratio_term(sj, dst));
    }
    double r;
    r = block_min(mp, sh); if (threadIdx.x == 0) part[0 * maxblk + blockIdx.x] = r;
    r = block_min(md, sh); if (threadIdx.x == 0) part[1 * maxblk + blockIdx.x] = r;
}

void ipm_recover_cc(hipStream_t st, const Red& r, int64_t n, const double* dw, const double* d,
                    const double* x, const double* s, double smu, double* dxa, double* dsa) {
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_recover_cc, dim3(nb), dim3(BLOCK), 0, st, n, dw, d, x, s, smu, dxa, dsa, r.part, r.maxblk);
    const int ops[2] = {1, 1};
    red_finish(st, r, 2, nb, ops);
}

__global__ __launch_bounds__(BLOCK) void k_ratio(int64_t n, const double* __restrict__ x,
                                                 const double* __restrict__ s,
                                                 const double* __restrict__ dx,
                                                 const double* __restrict__ ds,
                                                 double* __restrict__ part, int maxblk) {
    __shared__ double sh[BLOCK / 64];
    double mp = INFINITY, md = INFINITY;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += stride) {
        mp = fmin(mp, ratio_term(x[j], dx[j]));
        md = fmin(md, ratio_term(s[j], ds[j]));
    }
    double r;
    r = block_min(mp, sh); if (threadIdx.x == 0) part[0 * maxblk + blockIdx.x] = r;
    r = block_min(md, sh); if (threadIdx.x == 0) part[1 * maxblk + blockIdx.x] = r;
}

void ipm_ratio(hipStream_t st, const Red& r, int64_t n, const double* x, const double* s,
               const double* dx, const double* ds) {
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_ratio, dim3(nb), dim3(BLOCK), 0, st, n, x, s, dx, ds, r.part, r.maxblk);
    const int ops[2] = {1, 1};
    red_finish(st, r, 2, nb, ops);
}

// centrality test quantities at the trial point: min_i p_i and sum_i p_i,
// p_i = (x_i + ap dx_i)(s_i + ad ds_i)
__global__ __launch_bounds__(BLOCK) void k_backtrack(int64_t n, const double* __restrict__ x,
                                                     const double* __restrict__ s,
                                                     const double* __restrict__ dx,
                                                     const double* __restrict__ ds, double ap,
                                                     double ad, double* __restrict__ part,
                                                     int maxblk) {
    __shared__ double sh[BLOCK / 64];
    double mn = INFINITY, sm = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += stride) {
        const double p = (x[j] + ap * dx[j]) * (s[j] + ad * ds[j]);
        mn = fmin(mn, p);
        sm += p;
    }
    double r;
    r = block_min(mn, sh); if (threadIdx.x == 0) part[0 * maxblk + blockIdx.x] = r;
    r = block_sum(sm, sh); if (threadIdx.x == 0) part[1 * maxblk + blockIdx.x] = r;
}

void ipm_backtrack(hipStream_t st, const Red& r, int64_t n, const double* x, const double* s,
                   const double* dx, const double* ds, double ap, double ad) {
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_backtrack, dim3(nb), dim3(BLOCK), 0, st, n, x, s, dx, ds, ap, ad, r.part, r.maxblk);
    const int ops[2] = {1, 0};
    red_finish(st, r, 2, nb, ops);
}

// x += ap dx, s += ad ds, y += ad dy; count entries of x, s that are not finite positive
__global__ __launch_bounds__(BLOCK) void k_update(int64_t m, int64_t n, double* __restrict__ x,
                                                  double* __restrict__ s, double* __restrict__ y,
                                                  const double* __restrict__ dx,
                                                  const double* __restrict__ ds,
                                                  const double* __restrict__ dy, double ap,
                                                  double ad, double* __restrict__ part) {
    __shared__ double sh[BLOCK / 64];
    double bad = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += stride) {
        const double xn = x[j] + ap * dx[j];
        const double sn = s[j] + ad * ds[j];
        x[j] = xn;
        s[j] = sn;
        if (!(xn > 0.0) || !(sn > 0.0) || !isfinite(xn) || !isfinite(sn)) bad += 1.0;
    }
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < m; i += stride)
        y[i] = y[i] + ad * dy[i];
    const double r = block_sum(bad, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

void ipm_update(hipStream_t st, const Red& r, int64_t m, int64_t n, double* x, double* s,
                double* y, const double* dx, const double* ds, const double* dy, double ap,
                double ad) {
    const int nb = red_blocks(n > m ? n : m);
    hipLaunchKernelGGL(k_update, dim3(nb), dim3(BLOCK), 0, st, m, n, x, s, y, dx, ds, dy, ap, ad, r.part);
    const int ops[1] = {0};
    red_finish(st, r, 1, nb, ops);
}

// ------------------------------------------------------------------------------------
// small vector helpers
__global__ __launch_bounds__(BLOCK) void k_axpy(int64_t len, double a, const double* __restrict__ x,
                                                double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < len) y[i] = y[i] + a * x[i];
}
void axpy(hipStream_t st, int64_t len, double a, const double* x, double* y) {
    if (len > 0) hipLaunchKernelGGL(k_axpy, dim3(cdiv(len, BLOCK)), dim3(BLOCK), 0, st, len, a, x, y);
}

__global__ __launch_bounds__(BLOCK) void k_div_by(int64_t len, const double* __restrict__ a,
                                                  const double* __restrict__ rho,
                                                  double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < len) out[i] = a[i] / rho[i];
}
void div_by(hipStream_t st, int64_t len, const double* a, const double* rho, double* out) {
    if (len > 0) hipLaunchKernelGGL(k_div_by, dim3(cdiv(len, BLOCK)), dim3(BLOCK), 0, st, len, a, rho, out);
}

// dst[t] = src[perm[t]]
__global__ __launch_bounds__(BLOCK) void k_gather(int64_t len, const double* __restrict__ src,
                                                  const int32_t* __restrict__ perm,
                                                  double* __restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t < len) dst[t] = src[perm[t]];
}
void gather(hipStream_t st, int64_t len, const double* src, const int32_t* perm, double* dst) {
    if (len > 0) hipLaunchKernelGGL(k_gather, dim3(cdiv(len, BLOCK)), dim3(BLOCK), 0, st, len, src, perm, dst);
}
// dst[perm[t]] = src[t]
__global__ __launch_bounds__(BLOCK) void k_scatter(int64_t len, const double* __restrict__ src,
                                                   const int32_t* __restrict__ perm,
                                                   double* __restrict__ dst) {
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

// sum of squares of v into quantity 0 of r (then red_finish)
__global__ __launch_bounds__(BLOCK) void k_sumsq(int64_t len, const double* __restrict__ v,
                                                 double* __restrict__ part) {
    __shared__ double sh[BLOCK / 64];
    double q = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < len; i += stride) q += v[i] * v[i];
    const double r = block_sum(q, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}
void sumsq(hipStream_t st, const Red& r, int64_t len, const double* v) {
    const int nb = red_blocks(len);
    hipLaunchKernelGGL(k_sumsq, dim3(nb), dim3(BLOCK), 0, st, len, v, r.part);
    const int ops[1] = {0};
    red_finish(st, r, 1, nb, ops);
}

// v *= 1 / sqrt(out[0]) (after sumsq)
__global__ __launch_bounds__(BLOCK) void k_scale_by_norm(int64_t len, double* __restrict__ v,
                                                         const double* __restrict__ out) {
    const double nr = sqrt(out[0]);
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < len && nr > 0.0) v[i] = v[i] / nr;
}
void vec_scale_by_norm(hipStream_t st, const Red& r, int64_t len, double* v, int nblk_from) {
    (void)nblk_from;
    if (len > 0) hipLaunchKernelGGL(k_scale_by_norm, dim3(cdiv(len, BLOCK)), dim3(BLOCK), 0, st, len, v, r.out);
}

// out = a x + b y
__global__ __launch_bounds__(BLOCK) void k_lincomb(int64_t len, double a, const double* __restrict__ x,
                                                   double b, const double* __restrict__ y,
                                                   double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < len) out[i] = a * x[i] + b * y[i];
}
void lincomb(hipStream_t st, int64_t len, double a, const double* x, double b, const double* y,
             double* out) {
    if (len > 0) hipLaunchKernelGGL(k_lincomb, dim3(cdiv(len, BLOCK)), dim3(BLOCK), 0, st, len, a, x, b, y, out);
}

// starting point helpers: min x and min s
__global__ __launch_bounds__(BLOCK) void k_min2(int64_t n, const double* __restrict__ x,
                                                const double* __restrict__ s,
                                                double* __restrict__ part, int maxblk) {
    __shared__ double sh[BLOCK / 64];
    double a = INFINITY, b = INFINITY;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += stride) {
        const double xj = x[j], sj = s[j];
        a = fmin(a, isnan(xj) ? -INFINITY : xj);
        b = fmin(b, isnan(sj) ? -INFINITY : sj);
    }
    double r;
    r = block_min(a, sh); if (threadIdx.x == 0) part[0 * maxblk + blockIdx.x] = r;
    r = block_min(b, sh); if (threadIdx.x == 0) part[1 * maxblk + blockIdx.x] = r;
}
void min2(hipStream_t st, const Red& r, int64_t n, const double* x, const double* s) {
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_min2, dim3(nb), dim3(BLOCK), 0, st, n, x, s, r.part, r.maxblk);
    const int ops[2] = {1, 1};
    red_finish(st, r, 2, nb, ops);
}

// x += ax, s += as; then x.s, sum x, sum s
__global__ __launch_bounds__(BLOCK) void k_shift(int64_t n, double* __restrict__ x,
                                                 double* __restrict__ s, double ax, double as,
                                                 double* __restrict__ part, int maxblk) {
    __shared__ double sh[BLOCK / 64];
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += stride) {
        const double xj = x[j] + ax, sj = s[j] + as;
        x[j] = xj;
        s[j] = sj;
        q0 += xj * sj;
        q1 += xj;
        q2 += sj;
    }
    double r;
    r = block_sum(q0, sh); if (threadIdx.x == 0) part[0 * maxblk + blockIdx.x] = r;
    r = block_sum(q1, sh); if (threadIdx.x == 0) part[1 * maxblk + blockIdx.x] = r;
    r = block_sum(q2, sh); if (threadIdx.x == 0) part[2 * maxblk + blockIdx.x] = r;
}
void shift2(hipStream_t st, const Red& r, int64_t n, double* x, double* s, double ax, double as) {
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_shift, dim3(nb), dim3(BLOCK), 0, st, n, x, s, ax, as, r.part, r.maxblk);
    const int ops[3] = {0, 0, 0};
    red_finish(st, r, 3, nb, ops);
}

}  // namespace lpk
