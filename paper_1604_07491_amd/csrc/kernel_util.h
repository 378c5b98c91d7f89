// Device helpers shared by the kernel sources of the batched engine (gfx950, wave64):
// the instance/block map, sub-group and block reductions, reduction partials.  Not part of
// the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace lpk {

// The descriptors hold generic pointers; loads through them compile to flat accesses that
// wait on both memory counters.  Kernels view their global arrays through these casts so
// the loads are global loads and a batch of them can be in flight together.
#define LPK_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ LPK_GLOBAL T* to_global(T* p) { return (LPK_GLOBAL T*)p; }

// sum over k = s + lane, s + lane + g, ... < e of val[k] x[idx[k]], in increasing k.  The
// elements go in chunks of U per lane: the chunk's values and indices are loaded together,
// then its gathers of x, then the products are added (a lane past e adds zero terms).
template <int U, typename T>
__device__ __forceinline__ T row_dot(const LPK_GLOBAL T* __restrict__ val, const LPK_GLOBAL int32_t* __restrict__ idx,
                                     const LPK_GLOBAL T* __restrict__ x, int s, int e, int lane, int g) {
    T sum = 0;
    for (int kk = s + lane; kk < e; kk += U * g) {
        T v[U], xv[U];
        int j[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k2 = kk + u * g;
            const bool ok = k2 < e;
            v[u] = ok ? val[k2] : (T)0;
            j[u] = ok ? idx[k2] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = j[u] >= 0 ? x[j[u]] : (T)0;
#pragma unroll
        for (int u = 0; u < U; ++u) sum += v[u] * xv[u];
    }
    return sum;
}

constexpr int BLOCK = 256;
constexpr int GRID_CAP = 2048;

// Workgroups are dispatched to the 8 XCDs round-robin in linear order (x fastest).  When
// the batch is a multiple of 8, hardware block w is mapped to instance (w mod 8) + 8 q and
// block index w / 8 - q gx of it (q = (w / 8) / gx), so every block of one instance runs on
// the same XCD and that instance's vectors (z, V, the row data) stay in one L2.  Otherwise
// blockIdx is used as it is.  Either way the map is a bijection onto (instance, block).
struct BlockMap {
    int inst, bx;
};
__device__ __forceinline__ BlockMap block_map() {
    BlockMap r;
    const int gx = (int)gridDim.x;
    if ((gridDim.y & 7) == 0) {
        const int w = (int)blockIdx.x + (int)blockIdx.y * gx;
        const int local = w >> 3;
        const int q = local / gx;
        r.inst = (w & 7) + 8 * q;
        r.bx = local - q * gx;
    } else {
        r.inst = (int)blockIdx.y;
        r.bx = (int)blockIdx.x;
    }
    return r;
}

#define INST                               \
    const BlockMap bm_ = block_map();      \
    const int bx = bm_.bx;                 \
    (void)bx;                              \
    const Inst& in = I[bm_.inst]

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
static inline unsigned capg(int64_t blocks, int64_t cap) {
    if (blocks < 1) blocks = 1;
    return (unsigned)(blocks < cap ? blocks : cap);
}

// sum over a sub-group of g lanes (g a power of two <= 64)
template <typename T>
__device__ __forceinline__ T sg_sum(T v, int g) {
    for (int o = g >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, g);
    return v;
}

// sum over the lanes of a wave that agree in their low log2(il) bits (one interleaved row)
template <typename T>
__device__ __forceinline__ T il_sum(T v, int il) {
    for (int o = 32; o >= il; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// block-wide sum, valid on thread 0; sh holds blockDim.x / 64 doubles
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

__device__ __forceinline__ double block_min(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = INFINITY;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = fmin(r, sh[i]);
    return r;
}

__device__ __forceinline__ bool takes_part(const Inst& in, int pmask) {
    if (pmask > 0) return (*to_global(in.mode) & pmask) != 0;
    const LPK_GLOBAL KrylovCtl* ctl = to_global(in.ctl);
    if (pmask == PM_ITER_DIR) return ctl->done == 0 && ctl->cg_phase != 0;
    if (pmask == PM_NOKEEP) return ctl->done == 0 && in.keepz == 0;
    if (pmask == PM_NOFUSE) return ctl->done == 0 && in.fuse_u == 0;
    return ctl->done == 0;   // 0: Krylov loop, still iterating
}

// a launch of the sweep kernels in precision T serves only the instances whose sweeps run
// in that precision
template <typename T>
__device__ __forceinline__ bool other_precision(const Inst& in) {
    return (sizeof(T) == 4) != (in.fp32 != 0);
}

__device__ __forceinline__ void write_part(const Inst& in, int bx, int q, double v) {
    if (threadIdx.x == 0) to_global(in.part)[q * RED_MAXBLK + bx] = v;
}

}  // namespace lpk
