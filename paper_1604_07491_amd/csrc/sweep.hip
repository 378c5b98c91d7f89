// Inner-iteration sweeps of the batched engine on gfx950: the per-colour NE-SOR /
// NE-SSOR kernel (Sec. 3.3, 3.4 on the unit-row A_hat of Sec. 3.5).  Grid (x, S): one row
// of blocks per instance, as in kernels.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernel_util.h"
#include "kernels.h"

namespace lpk {

// ------------------------------------------------------------------------------------
// start of Krylov iteration k, NE-SOR instances whose colour 0 leaves some column
// uncovered: z = 0 (the first sweep sets V[:,k] and p_k itself)
__global__ __launch_bounds__(BLOCK) void k_prep(const Inst* __restrict__ I, int pmask) {
    INST;
    if (!takes_part(in, pmask) || in.gsor || in.zcover || in.lds || in.ncol == 0) return;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    if (in.fp32) {
        for (int64_t j = (int64_t)bx * BLOCK + threadIdx.x; j < in.n; j += stride) in.z32[j] = 0.0f;
    } else {
        double* __restrict__ z = in.vec[V_Z64];
        for (int64_t j = (int64_t)bx * BLOCK + threadIdx.x; j < in.n; j += stride) z[j] = 0.0;
    }
}

void b_prep(const BLaunch& L, int pmask) {
    hipLaunchKernelGGL(k_prep, dim3(capg(cdiv(L.max_n, BLOCK), GRID_CAP), L.S), dim3(BLOCK), 0, L.st, L.I, pmask);
}

// ------------------------------------------------------------------------------------
// One colour of a NE-SOR sweep (inner iteration of Sec. 3.4 on the unit-row A_hat): each
// row i of the colour, in parallel, computes d = omega (v_i - a_i . z), adds d to p_i and
// d a_i to z.  Rows of one colour share no column, so the z updates are disjoint.  The
// row segment (values, column indices) is held in registers between the dot product and
// the update, so each nonzero is read from memory once per sweep.  The loads go in three
// batches, each in flight together: the row's values and indices, then the gathers of z,
// then (after the sum) the stores of z; a lane past the row's end loads nothing and adds
// a zero term.  In FP64 (keepz) the
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
__global__ __launch_bounds__(BLOCK) void k_nesor(const Inst* __restrict__ I, int c, int sw, int npass, int dir, int keepz, int pmask, int ba) {
    INST;
    const LPK_GLOBAL KrylovCtl* ctl = to_global(in.ctl);
    if (!takes_part(in, pmask) || in.gsor || in.lds || c >= in.ncol || other_precision<T>(in)) return;
    if (in.cslice && to_global(in.cslice)[c] >= 0) return;   // a sliced colour (k_nesor_sl)
    const LPK_GLOBAL int32_t* cstart = to_global(in.cstart);
    const int r0 = cstart[c], r1 = cstart[c + 1], gc = to_global(in.cg)[c];
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
    const int write_z = (keepz && in.keepz) || !(sw == npass - 1 && c == (dir ? 0 : in.ncol - 1));
    // colour 0 of the first sweep reads z = 0 and overwrites its columns when it covers
    // every column (no clearing pass needed)
    const int fresh = sw == 0 && c == 0 && in.zcover;
    const int64_t k = ctl->k;
    // AB-GMRES / CG: input V_U / h into V[:,k], multipliers into P[:,k]; BA-GMRES: input
    // V_U as it is, kept in V_R64, multipliers into V_U
    LPK_GLOBAL double* __restrict__ vk = to_global(ba ? in.vec[V_R64] : in.V + k * in.ldv);
    LPK_GLOBAL double* __restrict__ p = to_global(ba ? in.vec[V_U] : in.P + k * in.ldv);
    const LPK_GLOBAL int32_t* __restrict__ rp = to_global(in.rp);
    const int s = rp[row], e = rp[row + 1];
    // first sweep: v_k = u / h_{k,k-1} is formed here and stored; p_k starts from delta
    const double vrow = sw == 0 ? to_global(in.vec[V_U])[row] * (ba ? 1.0 : ctl->inv_h) : vk[row];
    const LPK_GLOBAL T* __restrict__ val;
    LPK_GLOBAL T* __restrict__ z;
    if constexpr (sizeof(T) == 4) {
        val = to_global((const T*)in.ah32);
        z = to_global((T*)in.z32);
    } else {
        val = to_global((const T*)in.ah);
        z = to_global((T*)in.vec[V_Z64]);
    }
    const LPK_GLOBAL int32_t* __restrict__ idx = to_global(in.ci);
    T acc = 0;
    if (e - s <= g * R) {
        T a[R], zv[R];
        int j[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int kk = s + lane + t * g;
            const bool ok = kk < e;
            a[t] = ok ? val[kk] : (T)0;
            j[t] = ok ? idx[kk] : -1;
        }
#pragma unroll
        for (int t = 0; t < R; ++t) zv[t] = (!fresh && j[t] >= 0) ? z[j[t]] : (T)0;
#pragma unroll
        for (int t = 0; t < R; ++t) acc += a[t] * zv[t];
        acc = il ? il_sum(acc, il) : sg_sum(acc, g);
        const T delta = (T)in.omega * ((T)vrow - acc);
        if (write_z) {
#pragma unroll
            for (int t = 0; t < R; ++t)
                if (j[t] >= 0) z[j[t]] = fresh ? delta * a[t] : zv[t] + delta * a[t];
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

// ------------------------------------------------------------------------------------
// The same colour step on a sliced colour: a block of SL_THREADS threads takes a slice of
// SL_ROWS rows stored slot-major.  Thread (wave w, lane l) holds row r = l mod SL_ROWS and
// the slots s = 4 w + l / SL_ROWS + SL_GROUPS t, so a wave-wide load reads four whole slots,
// 64 consecutive values and indices; where the rows' columns advance together (the sinks
// of a transportation matrix) the z entries of a slot are neighbours too.  A row's sum adds
// the four slot groups of its wave (two butterfly steps), then the waves' partials in wave
// order.  Padding elements have column -1 and value 0.  Up to R slot steps per thread stay
// in registers (8, 12, 16 or 32: the fewest that hold the colour's longest slice, for
// occupancy); longer slices read their elements again for the z update.
static_assert(SL_ROWS == 16 && SL_THREADS % 64 == 0, "four slot groups per wave");

template <typename T, int R>
__global__ __launch_bounds__(SL_THREADS) void k_nesor_sl(const Inst* __restrict__ I, int c, int sw, int npass, int dir,
                                                         int keepz, int pmask, int ba) {
    __shared__ T red[SL_THREADS / 64][SL_ROWS];
    INST;
    const LPK_GLOBAL KrylovCtl* ctl = to_global(in.ctl);
    if (!takes_part(in, pmask) || in.gsor || in.lds || c >= in.ncol || !in.cslice || other_precision<T>(in)) return;
    const int q0 = to_global(in.cslice)[c];
    if (q0 < 0) return;
    const LPK_GLOBAL int32_t* cstart = to_global(in.cstart);
    const int r0 = cstart[c], r1 = cstart[c + 1];
    if (bx >= (r1 - r0 + SL_ROWS - 1) / SL_ROWS) return;   // the same for the whole block
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & (SL_ROWS - 1);
    const int grp = wv * (64 / SL_ROWS) + lane / SL_ROWS;
    const int row = r0 + bx * SL_ROWS + r;
    const bool live = row < r1;
    const int off = to_global(in.soff)[q0 + bx];
    const int steps = to_global(in.slen)[q0 + bx] / SL_GROUPS;
    const int write_z = (keepz && in.keepz) || !(sw == npass - 1 && c == (dir ? 0 : in.ncol - 1));
    const int fresh = sw == 0 && c == 0 && in.zcover;
    const int64_t k = ctl->k;
    LPK_GLOBAL double* __restrict__ vk = to_global(ba ? in.vec[V_R64] : in.V + k * in.ldv);
    LPK_GLOBAL double* __restrict__ p = to_global(ba ? in.vec[V_U] : in.P + k * in.ldv);
    double vrow = 0.0;
    if (live) vrow = sw == 0 ? to_global(in.vec[V_U])[row] * (ba ? 1.0 : ctl->inv_h) : vk[row];
    const LPK_GLOBAL T* __restrict__ val;
    LPK_GLOBAL T* __restrict__ z;
    if constexpr (sizeof(T) == 4) {
        val = to_global((const T*)in.sl_val32);
        z = to_global((T*)in.z32);
    } else {
        val = to_global((const T*)in.sl_val);
        z = to_global((T*)in.vec[V_Z64]);
    }
    const LPK_GLOBAL int32_t* __restrict__ idx = to_global(in.sl_idx);
    const int base = off + grp * SL_ROWS + r;   // slot grp of row r
    constexpr int STEP = SL_GROUPS * SL_ROWS;    // from one slot of the thread to its next
    const bool inreg = steps <= R;
    T acc = 0;
    T a[R], zv[R];
    int j[R];
    if (inreg) {
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const bool ok = t < steps;
            a[t] = ok ? val[base + t * STEP] : (T)0;
            j[t] = ok ? idx[base + t * STEP] : -1;
        }
#pragma unroll
        for (int t = 0; t < R; ++t) zv[t] = (!fresh && j[t] >= 0) ? z[j[t]] : (T)0;
#pragma unroll
        for (int t = 0; t < R; ++t) acc += a[t] * zv[t];
    } else if (!fresh) {
        for (int t = 0; t < steps; ++t) {
            const int jj = idx[base + t * STEP];
            if (jj >= 0) acc += val[base + t * STEP] * z[jj];
        }
    }
    acc += __shfl_xor(acc, 16, 64);
    acc += __shfl_xor(acc, 32, 64);
    if (lane < SL_ROWS) red[wv][lane] = acc;
    __syncthreads();
    T tot = 0;
#pragma unroll
    for (int w = 0; w < SL_THREADS / 64; ++w) tot += red[w][r];
    const T delta = (T)in.omega * ((T)vrow - tot);
    if (write_z) {
        if (inreg) {
#pragma unroll
            for (int t = 0; t < R; ++t)
                if (j[t] >= 0) z[j[t]] = fresh ? delta * a[t] : zv[t] + delta * a[t];
        } else {
            for (int t = 0; t < steps; ++t) {
                const int jj = idx[base + t * STEP];
                if (jj >= 0) {
                    const T av = val[base + t * STEP];
                    z[jj] = fresh ? delta * av : z[jj] + delta * av;
                }
            }
        }
    }
    if (wv == 0 && lane < SL_ROWS && live) {
        if (sw == 0) {
            vk[row] = vrow;
            p[row] = (double)delta;
        } else {
            p[row] += (double)delta;
        }
    }
}

// rows held in registers up to R elements per lane (8, 16 or 32: the most any instance
// needs for the colour; the arithmetic is the same for every R, only longer rows stream
// their elements twice)
template <typename T>
static void launch_nesor(const BLaunch& L, int R, dim3 gr, int colour, int pass, int npass, int dir, int kz,
                         int pmask) {
    const dim3 bl(BLOCK);
    const int ba = L.ba ? 1 : 0;
    if (R <= 8) hipLaunchKernelGGL((k_nesor<T, 8>), gr, bl, 0, L.st, L.I, colour, pass, npass, dir, kz, pmask, ba);
    else if (R <= 16) hipLaunchKernelGGL((k_nesor<T, 16>), gr, bl, 0, L.st, L.I, colour, pass, npass, dir, kz, pmask, ba);
    else hipLaunchKernelGGL((k_nesor<T, 32>), gr, bl, 0, L.st, L.I, colour, pass, npass, dir, kz, pmask, ba);
}

template <typename T>
static void launch_nesor_sl(const BLaunch& L, int R, dim3 gr, int colour, int pass, int npass, int dir, int kz,
                            int pmask) {
    const dim3 bl(SL_THREADS);
    const int ba = L.ba ? 1 : 0;
    if (R <= 8) hipLaunchKernelGGL((k_nesor_sl<T, 8>), gr, bl, 0, L.st, L.I, colour, pass, npass, dir, kz, pmask, ba);
    else if (R <= 12) hipLaunchKernelGGL((k_nesor_sl<T, 12>), gr, bl, 0, L.st, L.I, colour, pass, npass, dir, kz, pmask, ba);
    else if (R <= 16) hipLaunchKernelGGL((k_nesor_sl<T, 16>), gr, bl, 0, L.st, L.I, colour, pass, npass, dir, kz, pmask, ba);
    else hipLaunchKernelGGL((k_nesor_sl<T, 32>), gr, bl, 0, L.st, L.I, colour, pass, npass, dir, kz, pmask, ba);
}

// colour `colour` of every instance: the CSR launch for the instances that keep it in CSR
// form, the sliced launch for those that slice it (each kernel skips the other kind)
void b_nesor(const BLaunch& L, int colour, int pass, int npass, int dir, int pmask) {
    const int nc2 = L.max_ncol > 1 ? L.max_ncol : 1;
    // FP64 launches write z on the last colour for the instances that keep it (Inst::keepz)
    if (L.grid_colour[colour] > 0) {
        const dim3 gr(capg(L.grid_colour[colour], 1 << 30), L.S);
        const int R = L.colour_r[colour];
        if (L.any32) launch_nesor<float>(L, R, gr, colour, pass, npass, dir, 0, pmask);
        if (L.any64) launch_nesor<double>(L, R, gr, colour, pass, npass, dir, 1, pmask);
    }
    if (L.grid_colour[nc2 + colour] > 0) {
        const dim3 gr(capg(L.grid_colour[nc2 + colour], 1 << 30), L.S);
        const int R = L.colour_r[nc2 + colour];
        if (L.any32) launch_nesor_sl<float>(L, R, gr, colour, pass, npass, dir, 0, pmask);
        if (L.any64) launch_nesor_sl<double>(L, R, gr, colour, pass, npass, dir, 1, pmask);
    }
}

}  // namespace lpk
