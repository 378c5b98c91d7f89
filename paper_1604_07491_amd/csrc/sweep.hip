// Inner-iteration sweeps of the batched engine on gfx950: the per-colour NE-SOR /
// NE-SSOR kernel and the one-block LDS sweep for small LPs (Sec. 3.3, 3.4 on the unit-row
// A_hat of Sec. 3.5).  Grid (x, S): one row of blocks per instance, as in kernels.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernel_util.h"
#include "kernels.h"

namespace lpk {

// ------------------------------------------------------------------------------------
// start of Krylov iteration k, NE-SOR instances whose colour 0 leaves some column
// uncovered: z = 0 (the first sweep sets V[:,k] and p_k itself)
__global__ __launch_bounds__(BLOCK) void k_prep(const Inst* __restrict__ I, int mixed) {
    INST;
    if (in.ctl->done || in.gsor || in.zcover || in.lds || in.ncol == 0) return;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    if (mixed) {
        for (int64_t j = (int64_t)bx * BLOCK + threadIdx.x; j < in.n; j += stride) in.z32[j] = 0.0f;
    } else {
        double* __restrict__ z = in.vec[V_Z64];
        for (int64_t j = (int64_t)bx * BLOCK + threadIdx.x; j < in.n; j += stride) z[j] = 0.0;
    }
}

void b_prep(const BLaunch& L) {
    hipLaunchKernelGGL(k_prep, dim3(capg(cdiv(L.max_n, BLOCK), GRID_CAP), L.S), dim3(BLOCK), 0, L.st, L.I,
                       L.mixed);
}

// ------------------------------------------------------------------------------------
// One colour of a NE-SOR sweep (inner iteration of Sec. 3.4 on the unit-row A_hat): each
// row i of the colour, in parallel, computes d = omega (v_i - a_i . z), adds d to p_i and
// d a_i to z.  Rows of one colour share no column, so the z updates are disjoint.  The
// row segment (values, column indices) is held in registers between the dot product and
// the update, so each nonzero is read from memory once per sweep.  In FP64 (keepz) the
// last colour still updates z, which then holds z_k = A_hat^T p_k for the product that
// follows; in FP32 it skips the update and z_k is recomputed in FP64 from p.
//
// A pass visits the colours in order (dir 0) or in reverse (dir 1).  NE-SSOR (Sec. 3.3)
// alternates the two: each of its iterations is a forward and a backward sweep, and
// reversing the colour order reverses the row order of the colour-major permutation up to
// the order of rows inside one colour, which do not interact.
//
// Lanes of a row: cg[c] > 0: g = cg[c] consecutive lanes per row, a row's elements in
// lane order.  cg[c] < 0: interleaved, g = -cg[c] lanes per row spaced 64/g apart, so a
// wave holds 64/g consecutive rows and lanes with the same element slot sit next to each
// other.  The host picks per colour the form whose loads touch fewer cache lines (rows of
// a colour whose columns are strided, as the sinks of a transportation matrix, share
// lines across neighbouring rows).
template <typename T, int R>
__global__ __launch_bounds__(BLOCK) void k_nesor(const Inst* __restrict__ I, int c, int sw, int npass, int dir, int keepz) {
    INST;
    if (in.ctl->done || in.gsor || in.lds || c >= in.ncol) return;
    const int r0 = in.cstart[c], r1 = in.cstart[c + 1], gc = in.cg[c];
    const int tid = bx * BLOCK + threadIdx.x;
    int g, row, lane, il;
    if (gc > 0) {
        g = gc;
        il = 0;
        row = r0 + tid / g;
        lane = tid & (g - 1);
    } else {
        g = -gc;
        il = 64 / g;   // rows per wave
        const int w = tid >> 6, lw = tid & 63;
        row = r0 + w * il + (lw & (il - 1));
        lane = lw / il;
    }
    if (row >= r1) return;   // the same for every lane of the row; no block barrier below
    const int write_z = keepz || !(sw == npass - 1 && c == (dir ? 0 : in.ncol - 1));
    // colour 0 of the first sweep reads z = 0 and overwrites its columns when it covers
    // every column (no clearing pass needed)
    const int fresh = sw == 0 && c == 0 && in.zcover;
    const int64_t k = in.ctl->k;
    double* __restrict__ vk = in.V + k * in.ldv;
    double* __restrict__ p = in.P + k * in.ldv;
    // first sweep: v_k = u / h_{k,k-1} is formed here and stored; p_k starts from delta
    const double vrow = sw == 0 ? in.vec[V_U][row] * in.ctl->inv_h : vk[row];
    const T* __restrict__ val;
    T* __restrict__ z;
    if constexpr (sizeof(T) == 4) {
        val = (const T*)in.ah32;
        z = (T*)in.z32;
    } else {
        val = (const T*)in.ah;
        z = (T*)in.vec[V_Z64];
    }
    const int32_t* __restrict__ idx = in.ci;
    const int s = in.rp[row], e = in.rp[row + 1];
    T acc = 0;
    if (e - s <= g * R) {
        T a[R];
        int j[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int kk = s + lane + t * g;
            a[t] = 0;
            j[t] = 0;
            if (kk < e) {
                a[t] = val[kk];
                j[t] = idx[kk];
                if (!fresh) acc += a[t] * z[j[t]];
            }
        }
        acc = il ? il_sum(acc, il) : sg_sum(acc, g);
        const T delta = (T)in.omega * ((T)vrow - acc);
        if (write_z) {
#pragma unroll
            for (int t = 0; t < R; ++t)
                if (s + lane + t * g < e) {
                    if (fresh) z[j[t]] = delta * a[t];
                    else z[j[t]] += delta * a[t];
                }
        }
        if (lane == 0) {
            if (sw == 0) {
                vk[row] = vrow;
                p[row] = (double)delta;
            } else {
                p[row] += (double)delta;
            }
        }
    } else {
        if (!fresh)
            for (int kk = s + lane; kk < e; kk += g) acc += val[kk] * z[idx[kk]];
        acc = il ? il_sum(acc, il) : sg_sum(acc, g);
        const T delta = (T)in.omega * ((T)vrow - acc);
        if (write_z)
            for (int kk = s + lane; kk < e; kk += g) {
                if (fresh) z[idx[kk]] = delta * val[kk];
                else z[idx[kk]] += delta * val[kk];
            }
        if (lane == 0) {
            if (sw == 0) {
                vk[row] = vrow;
                p[row] = (double)delta;
            } else {
                p[row] += (double)delta;
            }
        }
    }
}

// rows held in registers up to R elements per lane: 8, or 16 when some instance lays the
// colour out interleaved (fewer lanes per row)
void b_nesor(const BLaunch& L, int colour, int pass, int npass, int dir) {
    const unsigned gx = capg(L.grid_colour[colour], 1 << 30);
    const bool wide = L.colour_il && L.colour_il[colour];
    const dim3 gr(gx, L.S), bl(BLOCK);
    const int kz = L.keep_z ? 1 : 0;
    if (L.mixed) {
        if (wide) hipLaunchKernelGGL((k_nesor<float, 16>), gr, bl, 0, L.st, L.I, colour, pass, npass, dir, 0);
        else hipLaunchKernelGGL((k_nesor<float, 8>), gr, bl, 0, L.st, L.I, colour, pass, npass, dir, 0);
    } else {
        if (wide) hipLaunchKernelGGL((k_nesor<double, 16>), gr, bl, 0, L.st, L.I, colour, pass, npass, dir, kz);
        else hipLaunchKernelGGL((k_nesor<double, 8>), gr, bl, 0, L.st, L.I, colour, pass, npass, dir, kz);
    }
}

// ------------------------------------------------------------------------------------
// A whole NE-SOR or NE-SSOR application (every pass over every colour) for instances
// whose z fits in LDS: one block of 1024 threads per instance, z zeroed and kept in LDS,
// a block barrier between colours instead of a kernel launch.  STAGED (Inst::lds == 2):
// the instance's whole row data (row pointers, values, column indices), v_k and the
// multipliers p_k are copied into LDS too, in one coalesced pass, so the colour steps,
// each a dependent chain of loads, run on LDS alone; v_k and p_k are written back at the
// end.  Each row is handled exactly as in k_nesor (same lanes per row, same
// element-to-lane assignment, same sub-group sum), so the result is bitwise the same as
// the per-colour launches.  keepz: z is copied out to V_Z64 at the end (z_k = A_hat^T p_k).  LDS layout (STAGED): p (m doubles), v (m doubles), values
// (nnz T), z (n T), row pointers (m + 1 ints), column indices (nnz ints).
constexpr int LDS_BLOCK = 1024;

template <typename T, bool STAGED>
__global__ __launch_bounds__(LDS_BLOCK) void k_sweep_lds(const Inst* __restrict__ I, int npass, int ssor, int keepz) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    INST;
    if (in.ctl->done || in.lds != (STAGED ? 2 : 1)) return;
    const int m = in.m, n = in.n, nnz = in.nnz;
    const int64_t k = in.ctl->k;
    const double ih = in.ctl->inv_h;
    const double* __restrict__ u = in.vec[V_U];
    double* __restrict__ vk = in.V + k * in.ldv;
    double* __restrict__ p = in.P + k * in.ldv;
    const T* __restrict__ gval;
    if constexpr (sizeof(T) == 4) gval = (const T*)in.ah32;
    else gval = (const T*)in.ah;
    T* __restrict__ z;
    const T* __restrict__ val;
    const int32_t* __restrict__ idx;
    const int32_t* __restrict__ rptr;
    double* __restrict__ pp;   // multipliers being accumulated
    double* __restrict__ vv;   // v_k as stored after the first pass
    if constexpr (STAGED) {
        double* pl = reinterpret_cast<double*>(lds_raw);
        double* vl = pl + m;
        T* sv = reinterpret_cast<T*>(vl + m);
        z = sv + nnz;
        int32_t* srp = reinterpret_cast<int32_t*>(z + n);
        int32_t* si = srp + (m + 1);
        for (int t = threadIdx.x; t < nnz; t += LDS_BLOCK) {
            sv[t] = gval[t];
            si[t] = in.ci[t];
        }
        for (int t = threadIdx.x; t <= m; t += LDS_BLOCK) srp[t] = in.rp[t];
        for (int t = threadIdx.x; t < m; t += LDS_BLOCK) vl[t] = u[t] * ih;
        val = sv;
        idx = si;
        rptr = srp;
        pp = pl;
        vv = vl;
    } else {
        z = reinterpret_cast<T*>(lds_raw);
        val = gval;
        idx = in.ci;
        rptr = in.rp;
        pp = p;
        vv = vk;
    }
    for (int j = threadIdx.x; j < n; j += LDS_BLOCK) z[j] = 0;
    __syncthreads();
    const T om = (T)in.omega;
    for (int sw = 0; sw < npass; ++sw) {
        const int dir = ssor ? (sw & 1) : 0;
        for (int cc = 0; cc < in.ncol; ++cc) {
            const int c = dir ? in.ncol - 1 - cc : cc;
            const int r0 = in.cstart[c], r1 = in.cstart[c + 1];
            const int g = in.cg[c] > 0 ? in.cg[c] : -in.cg[c];   // consecutive lanes here
            const int write_z = keepz || !(sw == npass - 1 && cc == in.ncol - 1);
            const int lane = threadIdx.x & (g - 1);
            const int per = LDS_BLOCK / g;
            for (int base = r0; base < r1; base += per) {
                const int row = base + (int)threadIdx.x / g;
                if (row < r1) {   // uniform inside the sub-group
                    const double vrow = (sw == 0 && !STAGED) ? u[row] * ih : vv[row];
                    const int s = rptr[row], e = rptr[row + 1];
                    constexpr int R = 8;
                    T acc = 0;
                    if (e - s <= g * R) {
                        T a[R];
                        int jj[R];
#pragma unroll
                        for (int t = 0; t < R; ++t) {
                            const int kk = s + lane + t * g;
                            a[t] = 0;
                            jj[t] = 0;
                            if (kk < e) {
                                a[t] = val[kk];
                                jj[t] = idx[kk];
                                acc += a[t] * z[jj[t]];
                            }
                        }
                        acc = sg_sum(acc, g);
                        const T delta = om * ((T)vrow - acc);
                        if (write_z) {
#pragma unroll
                            for (int t = 0; t < R; ++t)
                                if (s + lane + t * g < e) z[jj[t]] += delta * a[t];
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
                        acc = sg_sum(acc, g);
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
            __syncthreads();
        }
    }
    if constexpr (STAGED) {
        for (int t = threadIdx.x; t < m; t += LDS_BLOCK) {
            p[t] = pp[t];
            vk[t] = vv[t];
        }
    }
    if (keepz) {
        double* __restrict__ zo = in.vec[V_Z64];
        for (int j = threadIdx.x; j < n; j += LDS_BLOCK) zo[j] = (double)z[j];
    }
}

void b_sweep_lds(const BLaunch& L, int npass, int ssor, bool staged) {
    const dim3 gr(1, L.S), bl(LDS_BLOCK);
    const int by = staged ? L.stage_bytes : L.lds_bytes;
    const int kz = L.keep_z ? 1 : 0;
    if (staged) {
        if (L.mixed) hipLaunchKernelGGL((k_sweep_lds<float, true>), gr, bl, by, L.st, L.I, npass, ssor, 0);
        else hipLaunchKernelGGL((k_sweep_lds<double, true>), gr, bl, by, L.st, L.I, npass, ssor, kz);
    } else {
        if (L.mixed) hipLaunchKernelGGL((k_sweep_lds<float, false>), gr, bl, by, L.st, L.I, npass, ssor, 0);
        else hipLaunchKernelGGL((k_sweep_lds<double, false>), gr, bl, by, L.st, L.I, npass, ssor, kz);
    }
}

}  // namespace lpk
