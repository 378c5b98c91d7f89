// The one-block NE-SOR / NE-SSOR sweep of the batched engine for small LPs (Sec. 3.3, 3.4
// on the unit-row A_hat of Sec. 3.5), on gfx950.  Grid (1, S): one block per instance.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kernel_util.h"
#include "kernels.h"

namespace lpk {

// ------------------------------------------------------------------------------------
// A whole NE-SOR or NE-SSOR application (every pass over every colour) for instances
// whose z fits in LDS: one block of NT = 1024 threads per instance, z zeroed and kept in
// LDS, a block barrier between colours instead of a kernel launch.  v_k (formed from u at
// the start), the multipliers p_k and the row pointers sit in LDS too; the colour table
// (Inst::ctab) is read from device memory by scalar loads.  v_k and p_k are written back at the end.  STAGED (Inst::lds == 2): the row values and
// column indices are copied into LDS as well, in one coalesced pass, so the colour steps,
// each a dependent chain of loads, run on LDS alone; otherwise (Inst::lds == 1) they are
// read from memory (the instance's rows stay in the L2 cache over the passes).  A row takes
// its colour's lanes (at most LDS_LANES_MAX here when its longest row fits in LDS_SLOTS
// slots a lane), element kk on lane (kk - s) mod g in slot (kk - s) / g, each lane's
// elements summed in slot order, then the xor butterfly over the row's lanes.  keepz (Inst::keepz): z is copied out to V_Z64 at the end (z_k =
// A_hat^T p_k).  ba (BA-GMRES): the input is V_U as it is, kept in V_R64, and the
// multipliers go to V_U.  1024 threads per block measured as fast as 256 and twice as fast
// as 64 on the 200 x 500 LPs.
// LDS layout: p (m doubles), v (m doubles), [STAGED: values (nnz T)], z (n + 1 T: entry n
// takes the stores of the lanes past a row's end), row pointers (m + 1 ints), [STAGED:
// column indices (nnz ints)]: lds_stage_bytes / lds_z_bytes.  The colour table (first and
// last row, lanes per row, wave 0 alone, slots per lane) stays in device memory.
constexpr int NT = LDS_SWEEP_THREADS;

// one DPP lane move inside each row of 16 lanes (ctrl a quad_perm or row-mirror code)
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// v + (v of lane ^ 16) and v + (v of lane ^ 32) for every lane, by the gfx950 lane swaps:
// permlane16_swap(x, x) returns, in every lane, the even row's and the odd row's x of its
// pair of 16-lane rows, and permlane32_swap(x, x) the lower and the upper half's x of its
// lane (a 32-bit swap, applied to both halves of a double); their sum is the butterfly
// step's sum (addition commutes), with no LDS round trip.
__device__ __forceinline__ double xor16_add(double v) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ float xor16_add(float v) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double xor32_add(double v) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ float xor32_add(float v) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// sum over the g consecutive lanes of a row (g a power of two, the row's lanes all
// active).  Inside 16 lanes the partners come from DPP moves: quad_perm [1,0,3,2] and
// [2,3,0,1] (xor 1, xor 2), then the half-row and row mirrors, whose partners hold the
// same partial sums as the xor-4 and xor-8 partners; rows of 32 and 64 lanes finish with
// the lane swaps (xor 16, xor 32).  So the result is bitwise that of the xor butterfly,
// without an LDS round trip.
template <typename T>
__device__ __forceinline__ T sg_sum_lds(T v, int g) {
    if (g >= 2) v += dpp_move<0xB1>(v);
    if (g >= 4) v += dpp_move<0x4E>(v);
    if (g >= 8) v += dpp_move<0x141>(v);
    if (g >= 16) v += dpp_move<0x140>(v);
    if (g >= 32) v = xor16_add(v);
    if (g >= 64) v = xor32_add(v);
    return v;
}

// One row of a colour whose longest row needs at most S element slots per lane (S a
// compile-time count, so the loads are straight-line code with no branch between them):
// the row's values and indices are loaded together, then its z values; those are kept
// for the update: no other row of the colour touches these columns, so they are still
// current.  A slot past the row's end counts value 0 at the sink column n, whose z entry
// is 0 from the start and stays 0 (its updates add delta x 0): its term is +0, which
// leaves acc unchanged (it starts at +0 and never becomes -0), so the result does not
// depend on S beyond the row's need.  Its loads stay in bounds: in device memory at the
// row's last element; in LDS as they fall (an LDS read cannot fault, and its value is
// not used).  Returns the row's delta.
template <typename T, bool STAGED, int S>
__device__ __forceinline__ T row_step(const T* sv, const int32_t* si, const LPK_GLOBAL T* __restrict__ gval,
                                      const LPK_GLOBAL int32_t* __restrict__ gci, T* z, int n, int s, int e,
                                      int lane, int g, T om, double vrow, bool write_z) {
    T a[S], zv[S];
    int jj[S];
#pragma unroll
    for (int t = 0; t < S; ++t) {
        const int kk = s + lane + t * g;
        if constexpr (STAGED) {
            a[t] = sv[kk];
            jj[t] = si[kk];
        } else {
            const int kc = kk < e ? kk : e - 1;
            a[t] = gval[kc];
            jj[t] = gci[kc];
        }
    }
#pragma unroll
    for (int t = 0; t < S; ++t) {
        const bool ok = s + lane + t * g < e;
        a[t] = ok ? a[t] : (T)0;
        jj[t] = ok ? jj[t] : n;
        zv[t] = z[jj[t]];
    }
    T acc = 0;
#pragma unroll
    for (int t = 0; t < S; ++t) acc += a[t] * zv[t];
    acc = sg_sum_lds(acc, g);
    const T delta = om * ((T)vrow - acc);
    if (write_z) {
#pragma unroll
        for (int t = 0; t < S; ++t) z[jj[t]] = zv[t] + delta * a[t];
    }
    return delta;
}

template <typename T, bool STAGED>
__device__ __forceinline__ void sweep_lds_body(const Inst& in, unsigned char* lds_raw, int npass, int ssor, int ba,
                                               int fuse) {
    const int m = in.m, n = in.n, nnz = in.nnz, ncol = in.ncol;
    const int keepz = in.keepz;
    const int tid = threadIdx.x;
    const int64_t k = in.ctl->k;
    const double ih = ba ? 1.0 : in.ctl->inv_h;
    // global arrays through global-address-space pointers (global, not flat, loads)
    const LPK_GLOBAL double* __restrict__ u = to_global((const double*)in.vec[V_U]);
    double* __restrict__ vk = ba ? in.vec[V_R64] : in.V + k * in.ldv;
    double* __restrict__ p = ba ? in.vec[V_U] : in.P + k * in.ldv;
    const LPK_GLOBAL T* __restrict__ gval;
    if constexpr (sizeof(T) == 4) gval = to_global((const T*)in.ah32);
    else gval = to_global((const T*)in.ah);
    const LPK_GLOBAL int32_t* __restrict__ gci = to_global(in.ci);
    const LPK_GLOBAL int32_t* __restrict__ grp = to_global(in.rp);
    // the colour table (device memory, read-only): its entries are loaded by scalar loads
    const __attribute__((address_space(4))) int32_t* __restrict__ ctab =
        (const __attribute__((address_space(4))) int32_t*)in.ctab;
    double* pl = reinterpret_cast<double*>(lds_raw);   // multipliers being accumulated
    double* vl = pl + m;                               // v_k
    T* sv = reinterpret_cast<T*>(vl + m);              // STAGED: the row values
    T* z = STAGED ? sv + nnz : sv;
    int32_t* srp = reinterpret_cast<int32_t*>(z + n + 1);
    int32_t* si = srp + (m + 1);                       // STAGED: the column indices
    if constexpr (STAGED) {
#pragma unroll 4
        for (int t = tid; t < nnz; t += NT) {
            sv[t] = gval[t];
            si[t] = gci[t];
        }
    }
#pragma unroll 4
    for (int t = tid; t <= m; t += NT) srp[t] = grp[t];
#pragma unroll 4
    for (int t = tid; t < m; t += NT) vl[t] = u[t] * ih;
    for (int j = tid; j <= n; j += NT) z[j] = 0;
    __syncthreads();
    // A colour whose rows fit in one wave (rows x lanes <= 64) runs on wave 0 alone, and a
    // run of such colours needs no block barrier: the LDS accesses of one wave complete in
    // program order.
    const T om = (T)in.omega;
    constexpr int R = LDS_SLOTS;
    // A barrier precedes a whole-block colour that follows wave-0 colours and ends every
    // whole-block colour.
    bool prev_small = false;
    for (int sw = 0; sw < npass; ++sw) {
        const int dir = ssor ? (sw & 1) : 0;
        for (int cc = 0; cc < ncol; ++cc) {
            // the colour's entry, uniform: scalar registers, scalar branches
            const int c4 = 4 * (dir ? ncol - 1 - cc : cc);
            const int r0 = ctab[c4], r1 = ctab[c4 + 1], g = ctab[c4 + 2], cw = ctab[c4 + 3];
            const bool small = (cw & 1) != 0;
            const int slots = cw >> 1;   // element slots per lane of the colour's longest row
            const int write_z = keepz || !(sw == npass - 1 && cc == ncol - 1);
            const int lane = tid & (g - 1);
            const int lg = __builtin_ctz(g);   // g is a power of two
            if (!small && prev_small) __syncthreads();
            const int nth = small ? 64 : NT;
            const int per = nth >> lg;
            for (int base = r0; base < r1 && tid < nth; base += per) {
                const int row = base + (tid >> lg);
                if (row >= r1) continue;   // uniform inside the sub-group
                const double vrow = vl[row];
                const int s = srp[row], e = srp[row + 1];
                T acc = 0, delta;
                if (slots <= R) {
                    switch (slots) {
#define LPK_RS(S_)                                                                                    \
    case S_:                                                                                          \
        delta = row_step<T, STAGED, S_>(sv, si, gval, gci, z, n, s, e, lane, g, om, vrow, write_z != 0); \
        break;
                        LPK_RS(1) LPK_RS(2) LPK_RS(3) LPK_RS(4) LPK_RS(6) LPK_RS(8) LPK_RS(12) LPK_RS(16)
#undef LPK_RS
                        default: delta = 0; break;
                    }
                } else {
                    for (int kk = s + lane; kk < e; kk += g) {
                        if constexpr (STAGED) acc += sv[kk] * z[si[kk]];
                        else acc += gval[kk] * z[gci[kk]];
                    }
                    acc = sg_sum_lds(acc, g);
                    delta = om * ((T)vrow - acc);
                    if (write_z)
                        for (int kk = s + lane; kk < e; kk += g) {
                            if constexpr (STAGED) z[si[kk]] += delta * sv[kk];
                            else z[gci[kk]] += delta * gval[kk];
                        }
                }
                if (lane == 0) pl[row] = sw == 0 ? (double)delta : pl[row] + (double)delta;
            }
            if (!small) __syncthreads();
            prev_small = small;
        }
    }
    __syncthreads();   // the last colours may have run on wave 0 alone
    for (int t = tid; t < m; t += NT) {
        p[t] = pl[t];
        vk[t] = vl[t];
    }
    if (keepz) {
        double* __restrict__ zo = in.vec[V_Z64];
        for (int j = tid; j < n; j += NT) zo[j] = (double)z[j];
    }
    // AB-GMRES: u = A_hat z_k from the z this block holds, one row per thread, the row's
    // elements in index order (z is complete: keepz), instead of a product launch
    if (fuse && in.fuse_u) {
        LPK_GLOBAL double* __restrict__ uo = to_global(in.vec[V_U]);
        for (int row = tid; row < m; row += NT) {
            const int s = srp[row], e = srp[row + 1];
            double acc = 0.0;
            int kk = s;
            // eight elements' loads, then their gathers, then the products in index order
            for (; kk + 8 <= e; kk += 8) {
                T a[8], zv[8];
                int jj[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if constexpr (STAGED) {
                        a[q] = sv[kk + q];
                        jj[q] = si[kk + q];
                    } else {
                        a[q] = gval[kk + q];
                        jj[q] = gci[kk + q];
                    }
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) zv[q] = z[jj[q]];
#pragma unroll
                for (int q = 0; q < 8; ++q) acc += (double)a[q] * (double)zv[q];
            }
            for (; kk < e; ++kk) {
                if constexpr (STAGED) acc += (double)sv[kk] * (double)z[si[kk]];
                else acc += (double)gval[kk] * (double)z[gci[kk]];
            }
            uo[row] = acc;
        }
    }
}

// One launch serves every instance that sweeps from LDS, whatever its mode (STAGED or
// streamed) and precision: the branch is uniform per block, and separate launches per kind
// would run one after the other, each as long as its largest instance.
__global__ __launch_bounds__(NT) void k_sweep_lds(const Inst* __restrict__ I, int npass, int ssor, int pmask, int ba,
                                                  int fuse) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    INST;
    if (!takes_part(in, pmask) || in.lds == 0) return;
    if (in.fp32) {
        if (in.lds == 2) sweep_lds_body<float, true>(in, lds_raw, npass, ssor, ba, fuse);
        else sweep_lds_body<float, false>(in, lds_raw, npass, ssor, ba, fuse);
    } else {
        if (in.lds == 2) sweep_lds_body<double, true>(in, lds_raw, npass, ssor, ba, fuse);
        else sweep_lds_body<double, false>(in, lds_raw, npass, ssor, ba, fuse);
    }
}

void b_sweep_lds(const BLaunch& L, int npass, int ssor, int pmask, int fuse) {
    // LDS beyond 64 KiB per block is asked for once (gfx950: 160 KiB)
    static bool big_lds = false;
    if (!big_lds)
        big_lds = hipFuncSetAttribute((const void*)k_sweep_lds, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BLOCK_MAX) ==
                  hipSuccess;
    const int by = std::max(L.stage_bytes, L.lds_bytes);
    hipLaunchKernelGGL(k_sweep_lds, dim3(1, L.S), dim3(NT), by, L.st, L.I, npass, ssor, pmask, L.ba ? 1 : 0, fuse);
}

}  // namespace lpk
