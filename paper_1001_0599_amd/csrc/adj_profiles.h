// Pass 1 of the adjoint P^T (the exact transpose of the column-coherent trilinear P): the z
// profiles of one (view, detector column), one work-group per column.
//
// P sums, for every ray (view t, column i, row j) and sample k, w_ij * Lx Ly Lz f, with Lx Ly the
// bilinear weights of the sample's transverse position and Lz the linear weight of the row's z
// index s_kj = gamma_k q_j + (nz-1)/2.  Hence
//   (P^T y)_abc = sum_t sum_i sum_k Lx(a) Ly(b) Z_tik(c),  Z_tik(c) = sum_j w_ij y_tji hat(s_kj - c).
// The work-group forms FP64 prefix sums A[J] = sum_{j<J} W_j and B[J] = sum_{j<J} j W_j (W = w y)
// over the column's rows and writes Z_tik(c) for every sample k inside the grid's support and
// every cell c, each in O(1): the rows with s in [c-1, c) and [c, c+1) are the index ranges
// [J(c-1), J(c)) and [J(c), J(c+1)) with J(x) = ceil((x - (nz-1)/2)/gamma_k + (nv-1)/2), and the
// hat weights are linear in q_j on each range.  The profiles of a column are contiguous, cell
// index fastest.
#pragma once

#include <hip/hip_runtime.h>

#include "cbct_internal.h"

typedef float prof_v4f __attribute__((ext_vector_type(4)));  // a native vector for the non-temporal builtin

// The column's detector values are src[j * stride], j = 0 .. nv-1 (a projection column in global
// memory).  PREWEIGHTED: they are already w_ij * y.  ab: the LDS table, (nv + 1 + zk_max) double2
// when gb_lds, else (nv + 1).  Any block size that is a multiple of 64, up to 1024.
template <bool PREWEIGHTED>
__device__ __forceinline__ void column_profiles(const float *__restrict__ src, long stride, const ColParams cp,
                                                const ZIndex zi, int nv, int nz, float pv, bool gb_lds,
                                                float *__restrict__ Z, double2 *ab) {
    // ab: [nv + 1] (A, B), then [max nk] per-sample constants
    __shared__ double wtot[16][2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = (int)blockDim.x >> 6;
    const float iv = 0.5f * (float)(nv - 1);
    // prefix sums: rows in chunks of one row per thread, each chunk scanned by the block (wave
    // scans of 64 rows, then the earlier pieces' totals added in order: the sums depend on the
    // 64-row pieces only, not on the block size)
    double carry_a = 0.0, carry_b = 0.0;
    if (tid == 0) ab[0] = make_double2(0.0, 0.0);
    for (int j0 = 0; j0 < nv; j0 += (int)blockDim.x) {
        const int j = j0 + tid;
        double wa = 0.0, wb = 0.0;
        if (j < nv) {
            float w = src[(long)j * stride];
            const float q = (float)j - iv;
            if (!PREWEIGHTED) {
                const float v = q * pv;
                w *= cp.wsc * sqrtf(fmaf(v, v, cp.r2));
            }
            wa = (double)w;
            wb = (double)w * (double)j;  // exact: a float times an integer below 2^24
        }
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double ta = __shfl_up(wa, o), tb = __shfl_up(wb, o);
            if (lane >= o) {
                wa += ta;
                wb += tb;
            }
        }
        if (lane == 63) {
            wtot[wave][0] = wa;
            wtot[wave][1] = wb;
        }
        __syncthreads();
        double oa = carry_a, ob = carry_b;
        for (int w = 0; w < wave; w++) {
            oa += wtot[w][0];
            ob += wtot[w][1];
        }
        if (j < nv) ab[j + 1] = make_double2(oa + wa, ob + wb);
        for (int w = 0; w < nw; w++) {
            carry_a += wtot[w][0];
            carry_b += wtot[w][1];
        }
        __syncthreads();
    }
    // profiles: items (sample, CG consecutive cells), cells fastest.  With x_c = (c - beta) / gamma
    // + iv (cell c in row-index units) and S2(x) = sum_{j < x} W_j (x - j) = x A(J) - B(J), J = ceil(x)
    // the rows below x (clamped to [0, nv]), the hat sum is a second difference:
    //   Z(c) = sum_j W_j hat(gamma (q_j - x_c)) = gamma (S2(x_{c+1}) - 2 S2(x_c) + S2(x_{c-1})),
    // since x_{c+1} - x_c = 1 / gamma is the hat's half-width; CG + 2 evaluations of S2 (one prefix
    // lookup each) serve the item's CG cells.  The FP64 prefix sums keep the cancellation harmless
    // (|S2| is at most a few 1e5 times the row values).  CG = 4: each lane stores one float4, so
    // a wave's store covers 1 KB of consecutive profile floats; with CG = 8 (two float4 per lane,
    // 16-byte pieces at a 32-byte stride per store, 1.25 instead of 1.5 evaluations per cell) a P^T
    // at 512x512x64 / 40 views took 1.71-1.72 against 1.63 ms.
    constexpr int CG = 4;
    const double beta = 0.5 * (double)(nz - 1);
    const int nq = (nz + CG - 1) / CG;
    const bool vec = (nz & 3) == 0;
    float *zc = Z + zi.off;
    // per sample: 1 / gamma and iv - beta / gamma, once (an FP64 division is a long sequence),
    // when the column's samples fit in LDS
    double2 *gb = ab + (nv + 1);
    if (gb_lds) {
        for (int kk = tid; kk < zi.nk; kk += blockDim.x) {
            const double ig = 1.0 / (double)fmaf((float)(zi.k0 + kk), cp.dg, cp.g0);
            gb[kk] = make_double2(ig, (double)iv - beta * ig);
        }
        __syncthreads();
    }
    // items it = tid + m * blockDim: (kk, cq) advance by (dkk, dcq) with one carry (none when nq
    // divides the block size: then every thread keeps its cell group)
    const int dkk = (int)blockDim.x / nq, dcq = (int)blockDim.x - dkk * nq;
    int kk = tid / nq, cq = tid - kk * nq;
    for (; kk < zi.nk; kk += dkk, cq += dcq) {
        if (dcq != 0 && cq >= nq) {
            cq -= nq;
            if (++kk >= zi.nk) break;
        }
        const int cg0 = cq * CG;
        const double gamma = (double)fmaf((float)(zi.k0 + kk), cp.dg, cp.g0);
        double ig, base;
        if (gb_lds) {
            const double2 gbk = gb[kk];
            ig = gbk.x;
            base = gbk.y;
        } else {
            ig = 1.0 / gamma;
            base = (double)iv - beta * ig;
        }
        double s2[CG + 2];
        double xr = fma((double)(cg0 - 1), ig, base);  // x of cell cg0 - 1 (row-index units)
#pragma unroll
        for (int q = 0; q < CG + 2; q++) {
            if (q) xr += ig;
            const double2 p = ab[min(max((int)ceil(xr), 0), nv)];
            s2[q] = fma(xr, p.x, -p.y);
        }
        float o[CG];
#pragma unroll
        for (int q = 0; q < CG; q++) o[q] = (float)(gamma * fma(-2.0, s2[q + 1], s2[q] + s2[q + 2]));
        float *dst = zc + (long)kk * nz + cg0;
        if (vec && (CG & 3) == 0 && cg0 + CG <= nz) {
            // non-temporal: the gather reads these lines once, from HBM (P^T 1.50-1.52 against
            // 1.53-1.54 ms at the fine level, 0.26 against 0.27 ms at the coarse one)
#pragma unroll
            for (int q = 0; q < CG / 4; q++) {
                const prof_v4f t = {o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]};
                __builtin_nontemporal_store(t, reinterpret_cast<prof_v4f *>(dst + 4 * q));
            }
        } else {
#pragma unroll
            for (int q = 0; q < CG; q++)
                if (cg0 + q < nz) dst[q] = o[q];
        }
    }
}
