// The one-block NE-SOR / NE-SSOR sweep of the batched engine for small LPs (Sec. 3.3, 3.4
// on the unit-row A_hat of Sec. 3.5), on gfx950.  Grid (1, S): one block per instance.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernel_util.h"
#include "kernels.h"

namespace lpk {

// ------------------------------------------------------------------------------------
// A whole NE-SOR or NE-SSOR application (every pass over every colour) for instances
// whose z fits in LDS: one block of NT = 1024 threads per instance, z zeroed and kept in LDS,
// a block barrier between colours instead of a kernel launch.  The colour ranges and lanes
// are copied into LDS first.  STAGED (Inst::lds == 2): the instance's whole row data (row
// pointers, values, column indices), v_k and the multipliers p_k are copied into LDS too,
// in one coalesced pass, so the colour steps, each a dependent chain of loads, run on LDS
// alone; v_k and p_k are written back at the end.  Each row is handled exactly as in
// k_nesor (same lanes per row, same element-to-lane assignment, same sub-group sum).
// keepz: z is copied out to V_Z64 at the end (z_k = A_hat^T p_k).  ba (BA-GMRES): the
// input is V_U as it is, kept in V_R64, and the multipliers go to V_U.  A colour step is a
// chain of dependent LDS accesses, sub-group shuffles and a barrier; 1024 threads per block
// measured as fast as 256 and twice as fast as 64 on the 200 x 500 LPs.
// LDS layout (STAGED): p (m doubles), v (m doubles), values (nnz T), z (n T), row pointers
// (m + 1 ints), column indices (nnz ints), colour starts (ncol + 1 ints), lanes (ncol ints).
// Otherwise: z (n T), colour starts, lanes.
constexpr int NT = 1024;

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

// sum over the g consecutive lanes of a row (g a power of two, the row's lanes all
// active).  Inside 16 lanes the partners come from DPP moves: quad_perm [1,0,3,2] and
// [2,3,0,1] (xor 1, xor 2), then the half-row and row mirrors, whose partners hold the
// same partial sums as the xor-4 and xor-8 partners; so the result is bitwise that of the
// xor butterfly, without an LDS round trip per step.  Wider rows finish with shuffles.
template <typename T>
__device__ __forceinline__ T sg_sum_lds(T v, int g) {
    if (g >= 2) v += dpp_move<0xB1>(v);
    if (g >= 4) v += dpp_move<0x4E>(v);
    if (g >= 8) v += dpp_move<0x141>(v);
    if (g >= 16) v += dpp_move<0x140>(v);
    for (int o = 16; o < g; o <<= 1) v += __shfl_xor(v, o, g);
    return v;
}

template <typename T, bool STAGED>
__global__ __launch_bounds__(NT) void k_sweep_lds(const Inst* __restrict__ I, int npass, int ssor, int keepz, int pmask, int ba) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    INST;
    if (!takes_part(in, pmask) || in.lds != (STAGED ? 2 : 1)) return;
    const int m = in.m, n = in.n, nnz = in.nnz, ncol = in.ncol;
    const int64_t k = in.ctl->k;
    const double ih = ba ? 1.0 : in.ctl->inv_h;
    const double* __restrict__ u = in.vec[V_U];
    double* __restrict__ vk = ba ? in.vec[V_R64] : in.V + k * in.ldv;
    double* __restrict__ p = ba ? in.vec[V_U] : in.P + k * in.ldv;
    const T* __restrict__ gval;
    if constexpr (sizeof(T) == 4) gval = (const T*)in.ah32;
    else gval = (const T*)in.ah;
    T* __restrict__ z;
    const T* __restrict__ val;
    const int32_t* __restrict__ idx;
    const int32_t* __restrict__ rptr;
    int32_t* __restrict__ cs;  // colour starts
    int32_t* __restrict__ cl;  // lanes per row by colour
    double* __restrict__ pp;   // multipliers being accumulated
    double* __restrict__ vv;   // v_k as stored after the first pass
    if constexpr (STAGED) {
        double* pl = reinterpret_cast<double*>(lds_raw);
        double* vl = pl + m;
        T* sv = reinterpret_cast<T*>(vl + m);
        z = sv + nnz;
        int32_t* srp = reinterpret_cast<int32_t*>(z + n);
        int32_t* si = srp + (m + 1);
        cs = si + nnz;
        for (int t = threadIdx.x; t < nnz; t += NT) {
            sv[t] = gval[t];
            si[t] = in.ci[t];
        }
        for (int t = threadIdx.x; t <= m; t += NT) srp[t] = in.rp[t];
        for (int t = threadIdx.x; t < m; t += NT) vl[t] = u[t] * ih;
        val = sv;
        idx = si;
        rptr = srp;
        pp = pl;
        vv = vl;
    } else {
        z = reinterpret_cast<T*>(lds_raw);
        cs = reinterpret_cast<int32_t*>(z + n);
        val = gval;
        idx = in.ci;
        rptr = in.rp;
        pp = p;
        vv = vk;
    }
    cl = cs + (ncol + 1);
    for (int t = threadIdx.x; t <= ncol; t += NT) cs[t] = in.cstart[t];
    for (int t = threadIdx.x; t < ncol; t += NT) cl[t] = in.cg[t] > 0 ? in.cg[t] : -in.cg[t];   // consecutive lanes here
    for (int j = threadIdx.x; j < n; j += NT) z[j] = 0;
    __syncthreads();
    const T om = (T)in.omega;
    // A colour whose rows fit in one wave (rows x lanes <= 64) runs on wave 0 alone, and a
    // run of such colours needs no block barrier: the LDS accesses of one wave complete in
    // program order.  A barrier precedes a whole-block colour that follows wave-0 colours
    // and ends every whole-block colour.
    bool prev_small = false;
    for (int sw = 0; sw < npass; ++sw) {
        const int dir = ssor ? (sw & 1) : 0;
        for (int cc = 0; cc < ncol; ++cc) {
            const int c = dir ? ncol - 1 - cc : cc;
            const int r0 = cs[c], r1 = cs[c + 1];
            const int g = cl[c];
            const int write_z = keepz || !(sw == npass - 1 && cc == ncol - 1);
            const int lane = threadIdx.x & (g - 1);
            const bool small = (r1 - r0) * g <= 64;
            if (!small && prev_small) __syncthreads();
            const int nth = small ? 64 : NT;
            const int per = nth / g;
            for (int base = r0; base < r1 && (int)threadIdx.x < nth; base += per) {
                const int row = base + (int)threadIdx.x / g;
                if (row < r1) {   // uniform inside the sub-group
                    const double vrow = (sw == 0 && !STAGED) ? u[row] * ih : vv[row];
                    const int s = rptr[row], e = rptr[row + 1];
                    constexpr int R = 8;
                    T acc = 0;
                    if (e - s <= g * R) {
                        // (LDS loads return quickly; skipping the empty element slots by
                        // branch measured faster here than loading in batches).  The z
                        // values of the dot are kept for the update: no other row of the
                        // colour touches these columns, so they are still current.
                        T a[R], zv[R];
                        int jj[R];
#pragma unroll
                        for (int t = 0; t < R; ++t) {
                            const int kk = s + lane + t * g;
                            a[t] = 0;
                            zv[t] = 0;
                            jj[t] = 0;
                            if (kk < e) {
                                a[t] = val[kk];
                                jj[t] = idx[kk];
                                zv[t] = z[jj[t]];
                                acc += a[t] * zv[t];
                            }
                        }
                        acc = sg_sum_lds(acc, g);
                        const T delta = om * ((T)vrow - acc);
                        if (write_z) {
#pragma unroll
                            for (int t = 0; t < R; ++t)
                                if (s + lane + t * g < e) z[jj[t]] = zv[t] + delta * a[t];
                        }
                        if (lane == 0) {
                            if (sw == 0) {
                                if (!STAGED) vk[row] = vrow;
                                pp[row] = (double)delta;
                            } else {
                                pp[row] += (double)delta;
                            }
                        }
                    } else {
                        for (int kk = s + lane; kk < e; kk += g) acc += val[kk] * z[idx[kk]];
                        acc = sg_sum_lds(acc, g);
                        const T delta = om * ((T)vrow - acc);
                        if (write_z)
                            for (int kk = s + lane; kk < e; kk += g) z[idx[kk]] += delta * val[kk];
                        if (lane == 0) {
                            if (sw == 0) {
                                if (!STAGED) vk[row] = vrow;
                                pp[row] = (double)delta;
                            } else {
                                pp[row] += (double)delta;
                            }
                        }
                    }
                }
            }
            if (!small) __syncthreads();
            prev_small = small;
        }
    }
    __syncthreads();   // the last colours may have run on wave 0 alone
    if constexpr (STAGED) {
        for (int t = threadIdx.x; t < m; t += NT) {
            p[t] = pp[t];
            vk[t] = vv[t];
        }
    }
    if (keepz) {
        double* __restrict__ zo = in.vec[V_Z64];
        for (int j = threadIdx.x; j < n; j += NT) zo[j] = (double)z[j];
    }
}

void b_sweep_lds(const BLaunch& L, int npass, int ssor, bool staged, int pmask) {
    const dim3 gr(1, L.S), bl(NT);
    const int by = staged ? L.stage_bytes : L.lds_bytes;
    const int kz = L.keep_z ? 1 : 0, ba = L.ba ? 1 : 0;
    if (staged) {
        if (L.mixed) hipLaunchKernelGGL((k_sweep_lds<float, true>), gr, bl, by, L.st, L.I, npass, ssor, 0, pmask, ba);
        else hipLaunchKernelGGL((k_sweep_lds<double, true>), gr, bl, by, L.st, L.I, npass, ssor, kz, pmask, ba);
    } else {
        if (L.mixed) hipLaunchKernelGGL((k_sweep_lds<float, false>), gr, bl, by, L.st, L.I, npass, ssor, 0, pmask, ba);
        else hipLaunchKernelGGL((k_sweep_lds<double, false>), gr, bl, by, L.st, L.I, npass, ssor, kz, pmask, ba);
    }
}

}  // namespace lpk
