// Dense-panel path for problems created from a dense A (basis pursuit).
//
// Once per interior-point step the Gram matrix G = A_hat A_hat^T (m x m) of the unit-row
// A_hat is formed with FP64 matrix cores.  The inner iterations are then SOR on
// G p = v in natural row order, which in exact arithmetic is NE-SOR on the rows of A_hat
// (Sec. 3.4: the row update d_i = omega (g_i - alpha_i . z) with z = A_hat^T p is
// omega (g_i - G_i . p)), and the Krylov operator u = A_hat A_hat^T p is the product G p.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace lpk {

typedef double dbl4 __attribute__((ext_vector_type(4)));

static inline unsigned cdiv_u(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// ------------------------------------------------------------------------------------
// G = A A^T for a dense row-major A (m x n, leading dimension lda).  A block computes one
// 64 x 64 tile of the upper triangle (tile row bi <= tile column bj; the mirrored tile is
// written too, so G is exactly symmetric).  Each of the 4 waves owns a 32 x 32 quarter as
// 2 x 2 tiles of v_mfma_f64_16x16x4: lane l supplies a = A[r0 + l%16][k + l/16] and
// b = A[c0 + l%16][k + l/16]; result register r of lane l is D[l/16 + 4r][l%16].
// K is streamed in chunks of 32 through LDS; the next chunk's global loads are issued into
// registers before the current chunk's MFMAs, so they run under them.  With few tiles
// (m up to about 1,800) K is also split over blockIdx.y: each split writes its partial tile
// to a workspace and a second kernel adds the splits in a fixed order (deterministic).
constexpr int GT = 64;      // tile edge
constexpr int GKC = 32;     // k chunk staged in LDS
constexpr int GKP = GKC + 1;
constexpr int GLD = (GT * GKC) / 256;   // elements of a chunk each thread loads, per operand

static int gram_tiles(int m) {
    const int nb = (int)cdiv_u(m, GT);
    return nb * (nb + 1) / 2;
}

int gram_splits(int m) {
    const int t = gram_tiles(m);
    const int s = 1024 / t;
    return s < 1 ? 1 : (s > 8 ? 8 : s);
}

int64_t gram_work_doubles(int m) {
    const int s = gram_splits(m);
    return s > 1 ? (int64_t)s * gram_tiles(m) * GT * GT : 0;
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void k_gram(int m, int64_t n, const double* __restrict__ A, int64_t lda,
                                              double* __restrict__ G, float* __restrict__ G32,
                                              double* __restrict__ W, int nb, int ntile, int64_t kper) {
    // upper-triangle tile number -> (bi, bj), row by row
    int tl = blockIdx.x, bi = 0, rowlen = nb;
    while (tl >= rowlen) {
        tl -= rowlen;
        ++bi;
        rowlen = nb - bi;
    }
    const int bj = bi + tl;
    const int64_t kb = (int64_t)blockIdx.y * kper;
    const int64_t ke = kb + kper < n ? kb + kper : n;
    __shared__ double As[GT][GKP];
    __shared__ double Bs[GT][GKP];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;   // wave quarter inside the tile
    const int r0 = bi * GT, c0 = bj * GT;
    dbl4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
    double ra[GLD], rb[GLD];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < GLD; ++q) {
            const int e = tid + q * 256;
            const int rr = e / GKC, kk = e % GKC;
            const int64_t kg = k0 + kk;
            const int ia = r0 + rr, ib = c0 + rr;
            ra[q] = (ia < m && kg < ke) ? A[(int64_t)ia * lda + kg] : 0.0;
            rb[q] = (ib < m && kg < ke) ? A[(int64_t)ib * lda + kg] : 0.0;
        }
    };
    if (kb < ke) load(kb);
    for (int64_t k0 = kb; k0 < ke; k0 += GKC) {
#pragma unroll
        for (int q = 0; q < GLD; ++q) {
            const int e = tid + q * 256;
            As[e / GKC][e % GKC] = ra[q];
            Bs[e / GKC][e % GKC] = rb[q];
        }
        __syncthreads();
        if (k0 + GKC < ke) load(k0 + GKC);   // in flight during the MFMAs below
#pragma unroll
        for (int kk = 0; kk < GKC; kk += 4) {
            const int kl = kk + (lane >> 4);
            const double a0 = As[wr + (lane & 15)][kl];
            const double a1 = As[wr + 16 + (lane & 15)][kl];
            const double b0 = Bs[wc + (lane & 15)][kl];
            const double b1 = Bs[wc + 16 + (lane & 15)][kl];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int il = wr + 16 * a + (lane >> 4) + 4 * r;
                const int jl = wc + 16 * b + (lane & 15);
                const double v = acc[a][b][r];
                if constexpr (SPLIT) {
                    W[((int64_t)blockIdx.y * ntile + blockIdx.x) * (GT * GT) + il * GT + jl] = v;
                } else {
                    const int i = r0 + il, j = c0 + jl;
                    if (i < m && j < m) {
                        G[(int64_t)i * m + j] = v;
                        G[(int64_t)j * m + i] = v;
                        if (G32) {
                            G32[(int64_t)i * m + j] = (float)v;
                            G32[(int64_t)j * m + i] = (float)v;
                        }
                    }
                }
            }
}

// the splits of each tile added in split order, then written with the mirror; block
// (tile, y) takes the tile's elements [256 y, 256 y + 256)
__global__ __launch_bounds__(256) void k_gram_reduce(int m, const double* __restrict__ W, int nb, int ntile,
                                                     int splits, double* __restrict__ G, float* __restrict__ G32) {
    int tl = blockIdx.x, bi = 0, rowlen = nb;
    while (tl >= rowlen) {
        tl -= rowlen;
        ++bi;
        rowlen = nb - bi;
    }
    const int bj = bi + tl;
    {
        const int e = (int)blockIdx.y * 256 + threadIdx.x;
        double v = 0.0;
        for (int sp = 0; sp < splits; ++sp) v += W[((int64_t)sp * ntile + blockIdx.x) * (GT * GT) + e];
        const int i = bi * GT + e / GT, j = bj * GT + e % GT;
        if (i < m && j < m) {
            G[(int64_t)i * m + j] = v;
            G[(int64_t)j * m + i] = v;
            if (G32) {
                G32[(int64_t)i * m + j] = (float)v;
                G32[(int64_t)j * m + i] = (float)v;
            }
        }
    }
}

void gram_f64(hipStream_t st, int m, int64_t n, const double* A, int64_t lda, double* G, float* G32, double* W) {
    const int nb = (int)cdiv_u(m, GT), ntile = gram_tiles(m);
    const int splits = W ? gram_splits(m) : 1;
    const int64_t kper = ((n + splits - 1) / splits + GKC - 1) / GKC * GKC;
    if (splits > 1) {
        hipLaunchKernelGGL((k_gram<true>), dim3(ntile, splits), dim3(256), 0, st, m, n, A, lda, G, G32, W, nb,
                           ntile, kper);
        hipLaunchKernelGGL(k_gram_reduce, dim3(ntile, GT * GT / 256), dim3(256), 0, st, m, W, nb, ntile, splits, G,
                           G32);
    } else {
        hipLaunchKernelGGL((k_gram<false>), dim3(ntile, 1), dim3(256), 0, st, m, n, A, lda, G, G32, W, nb,
                           ntile, kper);
    }
}

// ------------------------------------------------------------------------------------
// D = alpha (A B) + beta E + F + diag_one * [row + r0 == col], all row-major (FP64
// MFMA, 64 x 64 tiles, k chunks of 32 staged in LDS, the next chunk loaded into registers
// under the current chunk's MFMAs).  A: M x K (lda), B: K x N (ldb).  E, F may be NULL.
// Used for the explicit inner-iteration preconditioner of the dense path.  With few tiles
// K is split over blockIdx.y into a workspace, and a second kernel adds the splits in order
// and applies the epilogue (deterministic).
__device__ __forceinline__ double gemm_epilogue(double acc, int i, int j, double alpha, double beta,
                                                const double* __restrict__ E, const double* __restrict__ F,
                                                int64_t lde, int diag_r0) {
    double v = alpha * acc;
    if (E) v += beta * E[(int64_t)i * lde + j];
    if (F) v += F[(int64_t)i * lde + j];
    if (diag_r0 >= 0 && i + diag_r0 == j) v += 1.0;
    return v;
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, double alpha,
                                              const double* __restrict__ A, int64_t lda,
                                              const double* __restrict__ B, int64_t ldb,
                                              double beta, const double* __restrict__ E,
                                              const double* __restrict__ F, int64_t lde,
                                              double* __restrict__ D, int64_t ldd, int diag_r0,
                                              int nbn, double* __restrict__ W, int kper) {
    __shared__ double As[GT][GKP];
    __shared__ double Bs[GT][GKP];   // Bs[col][k]
    const int bm = blockIdx.x / nbn, bn = blockIdx.x % nbn;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int r0 = bm * GT, c0 = bn * GT;
    const int kb = (int)blockIdx.y * kper;
    const int ke = kb + kper < K ? kb + kper : K;
    dbl4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
    double ra[GLD], rb[GLD];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < GLD; ++q) {
            const int e = tid + q * 256;
            // A tile: row rr, k kk (consecutive threads along k)
            const int rr = e / GKC, kk = e % GKC;
            const int ra_ = r0 + rr, ka = k0 + kk;
            ra[q] = (ra_ < M && ka < ke) ? A[(int64_t)ra_ * lda + ka] : 0.0;
            // B tile: k kb_, column cc (consecutive threads along the column)
            const int kb_ = e / GT, cc = e % GT;
            const int kg = k0 + kb_, cg = c0 + cc;
            rb[q] = (kg < ke && cg < N) ? B[(int64_t)kg * ldb + cg] : 0.0;
        }
    };
    if (kb < ke) load(kb);
    for (int k0 = kb; k0 < ke; k0 += GKC) {
#pragma unroll
        for (int q = 0; q < GLD; ++q) {
            const int e = tid + q * 256;
            As[e / GKC][e % GKC] = ra[q];
            Bs[e % GT][e / GT] = rb[q];
        }
        __syncthreads();
        if (k0 + GKC < ke) load(k0 + GKC);   // in flight during the MFMAs below
#pragma unroll
        for (int kk = 0; kk < GKC; kk += 4) {
            const int kl = kk + (lane >> 4);
            const double a0 = As[wr + (lane & 15)][kl];
            const double a1 = As[wr + 16 + (lane & 15)][kl];
            const double b0 = Bs[wc + (lane & 15)][kl];
            const double b1 = Bs[wc + 16 + (lane & 15)][kl];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
    const int ntile = (int)gridDim.x;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int il = wr + 16 * a + (lane >> 4) + 4 * r;
                const int jl = wc + 16 * b + (lane & 15);
                if constexpr (SPLIT) {
                    W[((int64_t)blockIdx.y * ntile + blockIdx.x) * (GT * GT) + il * GT + jl] = acc[a][b][r];
                } else {
                    const int i = r0 + il, j = c0 + jl;
                    if (i < M && j < N)
                        D[(int64_t)i * ldd + j] = gemm_epilogue(acc[a][b][r], i, j, alpha, beta, E, F, lde, diag_r0);
                }
            }
}

__global__ __launch_bounds__(256) void k_gemm_reduce(int M, int N, double alpha, double beta,
                                                     const double* __restrict__ E, const double* __restrict__ F,
                                                     int64_t lde, double* __restrict__ D, int64_t ldd,
                                                     int diag_r0, int nbn, const double* __restrict__ W,
                                                     int splits) {
    const int bm = blockIdx.x / nbn, bn = blockIdx.x % nbn;
    const int ntile = (int)gridDim.x;
    {   // block (tile, y) takes the tile's elements [256 y, 256 y + 256)
        const int e = (int)blockIdx.y * 256 + threadIdx.x;
        double acc = 0.0;
        for (int sp = 0; sp < splits; ++sp) acc += W[((int64_t)sp * ntile + blockIdx.x) * (GT * GT) + e];
        const int i = bm * GT + e / GT, j = bn * GT + e % GT;
        if (i < M && j < N) D[(int64_t)i * ldd + j] = gemm_epilogue(acc, i, j, alpha, beta, E, F, lde, diag_r0);
    }
}

void gemm_f64(hipStream_t st, int M, int N, int K, double alpha, const double* A, int64_t lda,
              const double* B, int64_t ldb, double beta, const double* E, const double* F,
              int64_t lde, double* D, int64_t ldd, int diag_r0, double* W, int64_t wcap) {
    if (M <= 0 || N <= 0) return;
    const int nbm = (int)cdiv_u(M, GT), nbn = (int)cdiv_u(N, GT);
    const int ntile = nbm * nbn;
    int splits = 1;
    if (W && K >= 8 * GKC) {
        splits = 512 / ntile;
        if (splits > 8) splits = 8;
        if (splits > K / (2 * GKC)) splits = K / (2 * GKC);
        while (splits > 1 && (int64_t)splits * ntile * GT * GT > wcap) --splits;
        if (splits < 1) splits = 1;
    }
    const int kper = ((K + splits - 1) / splits + GKC - 1) / GKC * GKC;
    if (splits > 1) {
        hipLaunchKernelGGL((k_gemm<true>), dim3(ntile, splits), dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb,
                           beta, E, F, lde, D, ldd, diag_r0, nbn, W, kper);
        hipLaunchKernelGGL(k_gemm_reduce, dim3(ntile, GT * GT / 256), dim3(256), 0, st, M, N, alpha, beta, E, F,
                           lde, D, ldd, diag_r0, nbn, W, splits);
    } else {
        hipLaunchKernelGGL((k_gemm<false>), dim3(ntile, 1), dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb,
                           beta, E, F, lde, D, ldd, diag_r0, nbn, W, kper);
    }
}

// Forward substitution with the diagonal block of M = I/omega + tril(G, -1) (rows
// [r0, r0+b) of the m x m G): X[r0 + i, j] = omega (R[i, j] - sum_{t<i} G[r0+i, r0+t] X[r0+t, j])
// for every column j < ncols; one thread per column, the block of G in LDS.
__global__ __launch_bounds__(256) void k_trsm_diag(int m, int r0, int b, const double* __restrict__ G,
                                                   const double* __restrict__ R, int64_t ldr,
                                                   double* __restrict__ X, double omega,
                                                   int ncols) {
    __shared__ double gb[64][65];
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int i = e / 64, t = e % 64;
        gb[i][t] = (i < b && t < b) ? G[(int64_t)(r0 + i) * m + r0 + t] : 0.0;
    }
    __syncthreads();
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= ncols) return;
    // the column of R is loaded first (its loads in flight together); the sum over t < i
    // runs on four accumulators (t mod 4) so that the FMAs of a row do not form one chain
    double x[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) x[i] = i < b ? R[(int64_t)i * ldr + j] : 0.0;
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        double s = 0.0;
        if (i < b) {
            double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < i; ++t) q[t & 3] += gb[i][t] * x[t];
            s = omega * (x[i] - ((q[0] + q[1]) + (q[2] + q[3])));
        }
        x[i] = s;
    }
#pragma unroll
    for (int i = 0; i < 64; ++i)
        if (i < b) X[(int64_t)(r0 + i) * m + j] = x[i];
}

void trsm_diag(hipStream_t st, int m, int r0, int b, const double* G, const double* R, int64_t ldr,
               double* X, double omega, int ncols) {
    if (ncols <= 0) return;
    hipLaunchKernelGGL(k_trsm_diag, dim3(cdiv_u(ncols, 256)), dim3(256), 0, st, m, r0, b, G, R, ldr, X, omega, ncols);
}

__global__ __launch_bounds__(256) void k_to_f32(int64_t len, const double* __restrict__ a, float* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) b[i] = (float)a[i];
}
void to_f32(hipStream_t st, int64_t len, const double* a, float* b) {
    if (len > 0) hipLaunchKernelGGL(k_to_f32, dim3(cdiv_u(len, 256)), dim3(256), 0, st, len, a, b);
}

}  // namespace lpk
