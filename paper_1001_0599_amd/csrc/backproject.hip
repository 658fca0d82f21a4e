// Adjoint P^T: the exact transpose of the forward projector, as a voxel-driven gather with
// no atomics (Section II.C.2 of the paper explains why a ray-driven scatter is a poor fit for
// GPUs: threads collide on voxels).
//
// P sums, for every ray (view t, column i, row j) and sample k, w_ij * Lx Ly Lz f, where Lx Ly
// are the bilinear weights of the sample's transverse position (shared by all rows of the
// column) and Lz the linear weight of the row's z index s_kj = gamma_k q_j + (nz-1)/2.  Hence
//   (P^T y)_abc = sum_t sum_i sum_k Lx(a) Ly(b) Z_tik(c),  Z_tik(c) = sum_j w_ij y_tji hat(s_kj - c).
//
// Two passes:
//  1. profiles: one work-group per (view, detector column) forms FP64 prefix sums
//     A[J] = sum_{j<J} W_j and B[J] = sum_{j<J} q_j W_j (W = w y) over the column's rows and
//     writes Z_tik(c) for every sample k inside the grid's support and every cell c, each in O(1):
//     the rows with s in [c-1, c) and [c, c+1) are the index ranges [J(c-1), J(c)) and
//     [J(c), J(c+1)) with J(x) = ceil((x - (nz-1)/2)/gamma_k + (nv-1)/2), and the hat weights are
//     linear in q_j on each range.  The profiles of a column are contiguous, cell index fastest.
//  2. gather: a work-group owns 16 x 16 voxel columns and up to 64 z cells and keeps its sums
//     in registers across all views; per view each voxel column visits the detector columns and
//     samples whose bilinear footprint covers it (exact windows) and adds Lx Ly times the
//     sample's profile segment (float4 loads, shared through the caches by neighbouring voxels).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <vector>

#include "cbct_internal.h"
#include "adj_profiles.h"

namespace {

// ---------------------------------------------------------------------------- pass 1
// PREWEIGHTED: the input already holds w_ij * y (the solver's residual epilogue writes it)
template <bool PREWEIGHTED>
__global__ void __launch_bounds__(512)
    k_adj_profiles(const float *__restrict__ proj, const ColParams *__restrict__ cols,
                   const ZIndex *__restrict__ zix, int nu, int nv, int nz, float pv, bool gb_lds,
                   float *__restrict__ Z) {
    extern __shared__ double2 ab[];
    // adjacent columns share the cache lines of their projection rows: keep them on one XCD
    const int w = cbct_xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int i = w % nu, view = w / nu;
    const long col = (long)view * nu + i;
    column_profiles<PREWEIGHTED>(proj + (long)view * nv * nu + i, nu, cols[col], zix[col], nv, nz, pv, gb_lds, Z, ab);
}

// ---------------------------------------------------------------------------- pass 2
// samples k of a column whose index coordinates lie in the open box (xa, xb) x (ya, yb),
// intersected with [lo, hi]; the caller takes klo = floor(lo) + 1, khi = ceil(hi) - 1.  A sample
// on the box boundary has interpolation weight 0 for the voxels inside.
__device__ __forceinline__ void window4(float fx0, float idfx, float fy0, float idfy, float xa, float xb, float ya,
                                        float yb, float &lo, float &hi) {
    if (idfx != 0.0f) {
        const float ka = (xa - fx0) * idfx, kb = (xb - fx0) * idfx;
        lo = fmaxf(lo, fminf(ka, kb));
        hi = fminf(hi, fmaxf(ka, kb));
    }
    if (idfy != 0.0f) {
        const float ka = (ya - fy0) * idfy, kb = (yb - fy0) * idfy;
        lo = fmaxf(lo, fminf(ka, kb));
        hi = fminf(hi, fmaxf(ka, kb));
    }
}

__device__ __forceinline__ void sample_window(const ColParams &cp, float xa, float xb, float ya, float yb, float &lo,
                                              float &hi) {
    window4(cp.fx0, cp.idfx, cp.fy0, cp.idfy, xa, xb, ya, yb, lo, hi);
}

// detector columns [i0, i1] whose rays cross the box [xa, xb] x [ya, yb] (mm, centred
// coordinates), widened by `widen` columns on each side: the central projections of the corners
// bound those of the whole box
__device__ __forceinline__ void box_columns(const AdjArgs &A, const ViewParams &vp, float xa, float xb, float ya,
                                            float yb, int widen, int &i0, int &i1) {
    float umin = FLT_MAX, umax = -FLT_MAX;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const float x = (q & 1) ? xb : xa, y = (q & 2) ? yb : ya;
        const float u = fmaf(x, vp.sn, -y * vp.cs) * A.sdd * __builtin_amdgcn_rcpf(fmaf(x, vp.cs, fmaf(y, vp.sn, A.sad)));
        umin = fminf(umin, u);
        umax = fmaxf(umax, u);
    }
    const float iu = 0.5f * (float)(A.nu - 1), ipu = 1.0f / A.pu;
    i0 = max(0, (int)ceilf(fmaf(umin, ipu, iu)) - widen);
    i1 = min(A.nu - 1, (int)floorf(fmaf(umax, ipu, iu)) + widen);
}

// Work-group -> tile: each XCD gets a contiguous band of tiles, whose neighbouring voxel
// columns read the same profiles through that XCD's L2.
__device__ __forceinline__ void tile_of(int &tx, int &ty, int &tz) {
    const int gx = gridDim.x, gy = gridDim.y;
    int w = cbct_xcd_remap(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    tx = w % gx;
    w /= gx;
    ty = w % gy;
    tz = w / gy;
}

template <int TZ, bool VEC>
__global__ void __launch_bounds__(256)
    k_adj_gather(const float *__restrict__ Z, const ZIndex *__restrict__ zix, const ColParams *__restrict__ cols,
                 const ViewParams *__restrict__ views, AdjArgs A, const float *__restrict__ fbase, float kappa,
                 float *__restrict__ out, int vgroups, int vper, float *__restrict__ part) {
    int tx, ty, tzg;
    tile_of(tx, ty, tzg);
    // view group g covers views [g vper, (g+1) vper) and writes part[g] (summed by k_adj_combine)
    const int nzt = (A.nz + TZ - 1) / TZ, tz = tzg % nzt, grp = tzg / nzt;
    const int v_begin = grp * vper, v_end = min(A.nviews, v_begin + vper);
    const int tid = threadIdx.x;
    const int a = tx * ADJ_TX + tid % ADJ_TX, b = ty * ADJ_TY + tid / ADJ_TX;
    const int c0 = tz * TZ;
    const float cx = 0.5f * (float)(A.nx - 1), cy = 0.5f * (float)(A.ny - 1);
    const float iu = 0.5f * (float)(A.nu - 1), ipu = 1.0f / A.pu;
    const float vx = ((float)a - cx) * A.hx, vy = ((float)b - cy) * A.hy;
    if (a >= A.nx || b >= A.ny) return;

    float acc[TZ];
#pragma unroll
    for (int q = 0; q < TZ; q++) acc[q] = 0.0f;

    for (int view = v_begin; view < v_end; view++) {
        const ViewParams vp = views[view];
        // detector columns whose samples can reach this voxel column: the footprint of its
        // support square (centre +- one voxel), widened by one column
        float umin = FLT_MAX, umax = -FLT_MAX;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float x = vx + ((q & 1) ? A.hx : -A.hx), y = vy + ((q & 2) ? A.hy : -A.hy);
            const float u = fmaf(x, vp.sn, -y * vp.cs) * A.sdd *
                            __builtin_amdgcn_rcpf(fmaf(x, vp.cs, fmaf(y, vp.sn, A.sad)));
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
        }
        const int i0 = max(0, (int)floorf(fmaf(umin, ipu, iu)) - 1);
        const int i1 = min(A.nu - 1, (int)ceilf(fmaf(umax, ipu, iu)) + 1);
        for (int i = i0; i <= i1; i++) {
            const long colx = (long)view * A.nu + i;
            const ColParams cp = cols[colx];
            const ZIndex zi = zix[colx];
            const float kb0 = (float)(zi.k0 - 1), kb1 = (float)(zi.k0 + zi.nk);
            float lo = kb0, hi = kb1;
            sample_window(cp, (float)(a - 1), (float)(a + 1), (float)(b - 1), (float)(b + 1), lo, hi);
            // clamp before the integer conversion (near-axis columns give huge window ends), which
            // keeps k inside [k0, k0 + nk - 1]
            lo = fminf(fmaxf(lo, kb0), kb1);
            hi = fminf(fmaxf(hi, kb0), kb1);
            const int klo = (int)floorf(lo) + 1, khi = min((int)ceilf(hi) - 1, zi.k0 + zi.nk - 1);
            for (int k = klo; k <= khi; k++) {
                const float kf = (float)k;
                const float fx = fmaf(kf, cp.dfx, cp.fx0), fy = fmaf(kf, cp.dfy, cp.fy0);
                const float wxy = fmaxf(1.0f - fabsf(fx - (float)a), 0.0f) * fmaxf(1.0f - fabsf(fy - (float)b), 0.0f);
                const float *zr = Z + zi.off + (long)(k - zi.k0) * A.nz + c0;
                if (VEC) {
#pragma unroll
                    for (int q = 0; q < TZ / 4; q++) {
                        const float4 z4 = *reinterpret_cast<const float4 *>(zr + 4 * q);
                        acc[4 * q + 0] = fmaf(wxy, z4.x, acc[4 * q + 0]);
                        acc[4 * q + 1] = fmaf(wxy, z4.y, acc[4 * q + 1]);
                        acc[4 * q + 2] = fmaf(wxy, z4.z, acc[4 * q + 2]);
                        acc[4 * q + 3] = fmaf(wxy, z4.w, acc[4 * q + 3]);
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < TZ; q++)
                        if (c0 + q < A.nz) acc[q] = fmaf(wxy, zr[q], acc[q]);
                }
            }
        }
    }
    const long nvox = (long)A.nx * A.ny * A.nz;
#pragma unroll
    for (int q = 0; q < TZ; q++) {
        const int c = c0 + q;
        if (c < A.nz) {
            const long idx = ((long)c * A.ny + b) * A.nx + a;
            if (vgroups > 1) part[grp * nvox + idx] = acc[q];
            else out[idx] = fbase ? fmaf(-kappa, acc[q], fbase[idx]) : acc[q];
        }
    }
}

// ---------------------------------------------------------------------------- pass 2, staged
// For nz a multiple of 32: a work-group owns 16 x 16 voxel columns x 32 z cells (one 128-byte
// line of every profile row).  Per view it lists the detector columns crossing its box and the
// samples of each inside the box (+ one voxel), stages those profile rows in LDS with coalesced
// loads (8 lanes per row), and every voxel column then gathers its hits from LDS.  Each profile
// line is read from L2 once per tile and view instead of once per voxel that uses it.
// Tiles of 32 z cells stage 320 rows per batch (52 KB of LDS: 3 work-groups per CU): on MI355X at
// 512x512x64 / 40 views in two view groups this measured 1.69-1.71 ms per P^T against 1.73-1.75
// for 288 rows and 1.80 for 224 or 256 (one view group: 288 was the fastest of 160 to 448), and
// tiles of 32 cells beat tiles of 64 (whole profile rows, 2 work-groups per CU: 2.16 against 1.99
// ms per P^T in one group).
constexpr int GS_ROWS32 = 320;
typedef float v4f __attribute__((ext_vector_type(4)));  // a native vector for the non-temporal builtin
constexpr int GS_CC = 64;  // detector columns per column chunk (one wave lists them)

struct GsCol {
    float fx0, dfx, fy0, dfy;  // index coordinates of sample k: (fx0 + k dfx, fy0 + k dfy)
    float idfx, idfy;          // samples per unit of x (of y); 0 when the column keeps x (y) fixed
    float hx, hy;              // |idfx| (|idfy|), or unbounded where that axis sets no window
    int ka, kb;                // samples of the column inside the tile box
    long zrow;                 // float offset of sample ka's cells c0.. in the profiles
};
static_assert(sizeof(GsCol) == 48, "GsCol layout");

template <int GS_TZ, int GS_ROWS>
struct GatherLds {
    static constexpr int PITCH = GS_TZ / 4 + 1;  // float4 slots per staged row (one pad slot)
    float4 zs[(GS_ROWS + 1) * PITCH];            // + one spill row for the staging's idle slots
    GsCol ci[GS_CC];
    int cnt[GS_CC + 1];    // exclusive row offsets of the chunk's columns; cnt[nc] = rows
    long rowsrc[GS_ROWS];  // profile offset of each staged row
};

// Tile (tx, ty, tz) of view group grp: the views [grp vper, (grp+1) vper).  With view groups
// (vgroups > 1) the sums go to part[grp] (k_adj_combine adds the groups in order); else
// out = fbase - kappa * sum (or the sum), and out2 the same when given.
template <int GS_TZ, int GS_ROWS>
__device__ __forceinline__ void gather_staged_body(GatherLds<GS_TZ, GS_ROWS> &lds, const float *__restrict__ Z,
                                                   const ZIndex *__restrict__ zix, const ColParams *__restrict__ cols,
                                                   const ViewParams *__restrict__ views, const AdjArgs &A, int tx,
                                                   int ty, int tz, int grp, int vgroups, int vper,
                                                   const float *__restrict__ fbase, float kappa,
                                                   float *__restrict__ out, float *__restrict__ out2,
                                                   float *__restrict__ part) {
    constexpr int GS_Q = GS_TZ / 4;             // float4 slots per profile row
    constexpr int GS_QS = GS_TZ == 64 ? 4 : 3;  // log2(GS_Q)
    constexpr int GS_PITCH = GS_Q + 1;
    float4 *zs = lds.zs;
    GsCol *ci = lds.ci;
    int *cnt = lds.cnt;
    long *rowsrc = lds.rowsrc;

    const int v_begin = grp * vper, v_end = min(A.nviews, v_begin + vper);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int a0 = tx * ADJ_TX, b0 = ty * ADJ_TY, c0 = tz * GS_TZ;
    const int a = a0 + (tid & (ADJ_TX - 1)), b = b0 + tid / ADJ_TX;
    const bool inside = a < A.nx && b < A.ny;
    const int alast = min(a0 + ADJ_TX - 1, A.nx - 1), blast = min(b0 + ADJ_TY - 1, A.ny - 1);
    const float cx = 0.5f * (float)(A.nx - 1), cy = 0.5f * (float)(A.ny - 1);
    // supports in mm: the tile's (union of the voxels' centre +- one voxel) and this voxel's
    const float txa = ((float)(a0 - 1) - cx) * A.hx, txb = ((float)(alast + 1) - cx) * A.hx;
    const float tya = ((float)(b0 - 1) - cy) * A.hy, tyb = ((float)(blast + 1) - cy) * A.hy;
    const float vxa = ((float)(a - 1) - cx) * A.hx, vxb = ((float)(a + 1) - cx) * A.hx;
    const float vya = ((float)(b - 1) - cy) * A.hy, vyb = ((float)(b + 1) - cy) * A.hy;

    float acc[GS_TZ];
#pragma unroll
    for (int q = 0; q < GS_TZ; q++) acc[q] = 0.0f;

    for (int view = v_begin; view < v_end; view++) {
        const ViewParams vp = views[view];
        int I0, I1, i0, i1;
        // the tile's list is widened so that it holds every column a voxel of the tile visits
        // (the voxel's exact range may round differently); a column whose ray only grazes a
        // support's edge carries weights of rounding size either way
        box_columns(A, vp, txa, txb, tya, tyb, 2, I0, I1);
        box_columns(A, vp, vxa, vxb, vya, vyb, 0, i0, i1);
        for (int cb = I0; cb <= I1; cb += GS_CC) {
            const int nc = min(GS_CC, I1 - cb + 1);
            // list the chunk's columns and their samples inside the tile box
            if (wave == 0) {
                int nr = 0;
                if (lane < nc) {
                    const long colx = (long)view * A.nu + cb + lane;
                    const ColParams cp = cols[colx];
                    const ZIndex zi = zix[colx];
                    const float kb0 = (float)(zi.k0 - 1), kb1 = (float)(zi.k0 + zi.nk);
                    float lo = kb0, hi = kb1;
                    sample_window(cp, (float)(a0 - 1), (float)(alast + 1), (float)(b0 - 1), (float)(blast + 1), lo,
                                  hi);
                    lo = fminf(fmaxf(lo, kb0), kb1);
                    hi = fminf(fmaxf(hi, kb0), kb1);
                    const int ka = (int)floorf(lo) + 1, kb = min((int)ceilf(hi) - 1, zi.k0 + zi.nk - 1);
                    nr = max(kb - ka + 1, 0);
                    GsCol g;
                    g.fx0 = cp.fx0;
                    g.dfx = cp.dfx;
                    g.fy0 = cp.fy0;
                    g.dfy = cp.dfy;
                    g.idfx = cp.idfx;
                    g.idfy = cp.idfy;
                    g.hx = cp.idfx != 0.0f ? fabsf(cp.idfx) : 1e30f;
                    g.hy = cp.idfy != 0.0f ? fabsf(cp.idfy) : 1e30f;
                    g.ka = ka;
                    g.kb = ka + nr - 1;
                    g.zrow = zi.off + (long)(ka - zi.k0) * A.nz + c0;
                    ci[lane] = g;
                }
                int incl = nr;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int t = __shfl_up(incl, o);
                    if (lane >= o) incl += t;
                }
                if (lane < nc) cnt[lane + 1] = incl;
                if (lane == 0) cnt[0] = 0;
            }
            __syncthreads();
            const int total = cnt[nc];
            // this voxel column's columns within the chunk
            const int t_lo = max(i0 - cb, 0), t_hi = min(i1 - cb, nc - 1);
            for (int R0 = 0; R0 < total; R0 += GS_ROWS) {
                const int nrows = min(GS_ROWS, total - R0);
                // profile offsets of this batch's rows
                // four threads per column (a chunk holds at most 64)
                if (tid < 4 * nc) {
                    const int t = tid >> 2;
                    const int r_a = max(cnt[t], R0), r_b = min(cnt[t + 1], R0 + nrows);
                    const long z0 = ci[t].zrow - (long)cnt[t] * A.nz;
                    for (int r = r_a + (tid & 3); r < r_b; r += 4) rowsrc[r - R0] = z0 + (long)r * A.nz;
                }
                __syncthreads();
                // stage the rows: 8 lanes per 128-byte row; every load of the batch is issued
                // before the first LDS store, so the batch pays one memory latency
                {
                    constexpr int PER = (GS_ROWS * GS_Q + 255) / 256;
                    const int items = nrows * GS_Q;  // > 0
                    static_assert(PER == 10, "the asm statement below lists the batch's ten loads");
                    v4f v[PER];
                    const float *zq = Z + 4 * (tid & (GS_Q - 1));  // this thread's float4 slot of a row
#pragma unroll
                    for (int j = 0; j < PER; j++) {
                        // item tid + 256 j: row (tid >> GS_QS) + j 256 / GS_Q; items past the batch load
                        // its last row again (no branch between the loads)
                        const int r = min((tid >> GS_QS) + j * (256 >> GS_QS), nrows - 1);
                        // a non-temporal load: these profile lines are read once, from HBM
                        v[j] = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(zq + rowsrc[r]));
                    }
                    // all loads in flight before the first store: an empty asm statement takes every
                    // loaded vector as an operand (no instructions), so the compiler cannot sink (or
                    // split) each load down to its store; idle slots store into the spill row
                    asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]),
                                 "v"(v[7]), "v"(v[8]), "v"(v[9]));
                    v4f *zsv = reinterpret_cast<v4f *>(zs);
#pragma unroll
                    for (int j = 0; j < PER; j++) {
                        const int it = tid + 256 * j;
                        const int r = it < items ? (it >> GS_QS) : GS_ROWS;
                        zsv[r * GS_PITCH + (it & (GS_Q - 1))] = v[j];
                    }
                }
                __syncthreads();
                if (inside) {
                    for (int t = t_lo; t <= t_hi; t++) {
                        const GsCol g = ci[t];
                        // staged samples of column t in this batch
                        const int kfirst = max(g.ka, g.ka + R0 - cnt[t]);
                        const int klast = min(g.kb, g.ka + R0 + nrows - 1 - cnt[t]);
                        const float kb0 = (float)(kfirst - 1), kb1 = (float)(klast + 1);
                        // samples within one voxel of (a, b): |k - kc| < h on each axis, kc the sample
                        // index at the voxel centre (a window-free axis has kc = 0, h unbounded)
                        const float fxa = g.fx0 - (float)a, fya = g.fy0 - (float)b;  // sample 0 relative to (a, b)
                        const float kcx = -fxa * g.idfx, kcy = -fya * g.idfy;
                        float lo = fmaxf(kcx - g.hx, kcy - g.hy), hi = fminf(kcx + g.hx, kcy + g.hy);
                        lo = fminf(fmaxf(lo, kb0), kb1);
                        hi = fminf(fmaxf(hi, kb0), kb1);
                        const int klo = (int)floorf(lo) + 1, khi = min((int)ceilf(hi) - 1, klast);
                        const int rbase = cnt[t] - R0 - g.ka;  // staged row of sample k: rbase + k
                        for (int k = klo; k <= khi; k++) {
                            const float kf = (float)k;
                            const float dx = fmaf(kf, g.dfx, fxa), dy = fmaf(kf, g.dfy, fya);
                            const float wxy = fmaxf(1.0f - fabsf(dx), 0.0f) * fmaxf(1.0f - fabsf(dy), 0.0f);
                            const float4 *zr = zs + (rbase + k) * GS_PITCH;
#pragma unroll
                            for (int q = 0; q < GS_Q; q++) {
                                const float4 z4 = zr[q];
                                acc[4 * q + 0] = fmaf(wxy, z4.x, acc[4 * q + 0]);
                                acc[4 * q + 1] = fmaf(wxy, z4.y, acc[4 * q + 1]);
                                acc[4 * q + 2] = fmaf(wxy, z4.z, acc[4 * q + 2]);
                                acc[4 * q + 3] = fmaf(wxy, z4.w, acc[4 * q + 3]);
                            }
                        }
                    }
                }
                __syncthreads();
            }
            // every wave has read this chunk's list before the next chunk overwrites it (also when
            // it had no rows, so no batch barrier ran)
            __syncthreads();
        }
    }
    if (inside) {
        const long nvox = (long)A.nx * A.ny * A.nz;
#pragma unroll
        for (int q = 0; q < GS_TZ; q++) {
            const long idx = ((long)(c0 + q) * A.ny + b) * A.nx + a;
            if (vgroups > 1) {
                part[grp * nvox + idx] = acc[q];
            } else {
                const float o = fbase ? fmaf(-kappa, acc[q], fbase[idx]) : acc[q];
                out[idx] = o;
                if (out2) out2[idx] = o;
            }
        }
    }
}

// grid (tiles x, tiles y, (nz / GS_TZ) * vgroups)
template <int GS_TZ, int GS_ROWS>
__global__ void __launch_bounds__(256)
    k_adj_gather_staged(const float *__restrict__ Z, const ZIndex *__restrict__ zix,
                        const ColParams *__restrict__ cols, const ViewParams *__restrict__ views, AdjArgs A,
                        int vgroups, int vper, const float *__restrict__ fbase, float kappa, float *__restrict__ out,
                        float *__restrict__ out2, float *__restrict__ part) {
    __shared__ GatherLds<GS_TZ, GS_ROWS> lds;
    int tx, ty, tzg;
    tile_of(tx, ty, tzg);
    const int nzt = A.nz / GS_TZ;
    gather_staged_body<GS_TZ, GS_ROWS>(lds, Z, zix, cols, views, A, tx, ty, tzg % nzt, tzg / nzt, vgroups, vper, fbase,
                                       kappa, out, out2, part);
}

// out = sum of the view groups' partial volumes (in group order), or fbase - kappa * that sum;
// also into out2 when given (the solver's ROF start u = g, saving a copy pass)
__global__ void __launch_bounds__(256) k_adj_combine(const float *__restrict__ part, int vgroups, long n,
                                                     const float *__restrict__ fbase, float kappa,
                                                     float *__restrict__ out, float *__restrict__ out2) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        float s = part[i];
        for (int g = 1; g < vgroups; g++) s += part[g * n + i];
        const float v = fbase ? fmaf(-kappa, s, fbase[i]) : s;
        out[i] = v;
        if (out2) out2[i] = v;
    }
}

// ---------------------------------------------------------------------------- batched (serving)
// Several requests in one launch: request q owns work-groups [wg0[q], wg0[q+1]) and each runs the
// solo kernel's body on that request's buffers, so the results are bitwise those of solo launches.
__device__ __forceinline__ int batch_item(const int *wg0, int n) {
    int r = 0;
    while (r + 1 < n && (int)blockIdx.x >= wg0[r + 1]) r++;
    return r;
}

struct BPrItem {  // profiles: one work-group per (view, column)
    const float *proj;
    const ColParams *cols;
    const ZIndex *zix;
    float *Z;
    int nu, nv, nz, nviews, gb_lds;
    float pv;
};
struct BPr {
    int n;
    int wg0[CBCT_MAXB + 1];
    BPrItem it[CBCT_MAXB];
};
__global__ void __launch_bounds__(256) k_adj_profiles_b(BPr B) {
    extern __shared__ double2 ab[];
    const int r = batch_item(B.wg0, B.n);
    const BPrItem &it = B.it[r];
    const int w = cbct_batch_local(B.wg0[r], B.wg0[r + 1] - B.wg0[r]);
    if (w >= it.nu * it.nviews) return;  // padding
    const int i = w % it.nu, view = w / it.nu;
    const long col = (long)view * it.nu + i;
    column_profiles<true>(it.proj + (long)view * it.nv * it.nu + i, it.nu, it.cols[col], it.zix[col], it.nv, it.nz,
                          it.pv, it.gb_lds != 0, it.Z, ab);
}

struct BGaItem {  // staged gather: one work-group per (tile, view group)
    const float *Z;
    const ZIndex *zix;
    const ColParams *cols;
    const ViewParams *views;
    const float *fbase;
    float *out, *out2, *part;
    AdjArgs A;
    int ntx, nty, vgroups, vper;
    float kappa;
};
struct BGa {
    int n;
    int wg0[CBCT_MAXB + 1];
    BGaItem it[CBCT_MAXB];
};
static_assert(sizeof(BGa) <= 4096, "batched gather arguments");
__global__ void __launch_bounds__(256) k_adj_gather_staged_b(BGa B) {
    __shared__ GatherLds<32, GS_ROWS32> lds;
    const int r = batch_item(B.wg0, B.n);
    const BGaItem &it = B.it[r];
    const int nzt = it.A.nz / 32;
    const int w = cbct_batch_local(B.wg0[r], B.wg0[r + 1] - B.wg0[r]);
    if (w >= it.ntx * it.nty * nzt * it.vgroups) return;  // padding
    const int tzg = w / (it.ntx * it.nty), t2 = w - tzg * it.ntx * it.nty;
    gather_staged_body<32, GS_ROWS32>(lds, it.Z, it.zix, it.cols, it.views, it.A, t2 % it.ntx, t2 / it.ntx, tzg % nzt,
                                      tzg / nzt, it.vgroups, it.vper, it.fbase, it.kappa, it.out, it.out2, it.part);
}

struct BCoItem {  // view-group sums: nb work-groups striding over the request's voxels
    const float *part;
    const float *fbase;
    float *out, *out2;
    long n;
    int vgroups;
    float kappa;
};
struct BCo {
    int n;
    int wg0[CBCT_MAXB + 1];
    BCoItem it[CBCT_MAXB];
};
__global__ void __launch_bounds__(256) k_adj_combine_b(BCo B) {
    const int r = batch_item(B.wg0, B.n);
    const BCoItem &it = B.it[r];
    const long w = (long)blockIdx.x - B.wg0[r], nb = B.wg0[r + 1] - B.wg0[r];
    for (long i = w * blockDim.x + threadIdx.x; i < it.n; i += nb * blockDim.x) {
        float s = it.part[i];
        for (int g = 1; g < it.vgroups; g++) s += it.part[g * it.n + i];
        const float v = it.fbase ? fmaf(-it.kappa, s, it.fbase[i]) : s;
        it.out[i] = v;
        if (it.out2) it.out2[i] = v;
    }
}

#define LAUNCH_CHECK(what)                                     \
    do {                                                       \
        hipError_t e_ = hipGetLastError();                     \
        if (e_ != hipSuccess) return cbct_hip_error(e_, what); \
    } while (0)

template <int TZ>
cbct_status launch_gather(const Level &L, const float *Z, const float *fbase, float kappa, float *out, int vg,
                          int vper, float *part, hipStream_t s) {
    dim3 grid((L.nx + ADJ_TX - 1) / ADJ_TX, (L.ny + ADJ_TY - 1) / ADJ_TY, ((L.nz + TZ - 1) / TZ) * vg);
    if (L.nz % TZ == 0)
        hipLaunchKernelGGL((k_adj_gather<TZ, true>), grid, dim3(ADJ_TX * ADJ_TY), 0, s, Z, L.d_zix, L.d_cols,
                           L.d_views, L.adj, fbase, kappa, out, vg, vper, part);
    else
        hipLaunchKernelGGL((k_adj_gather<TZ, false>), grid, dim3(ADJ_TX * ADJ_TY), 0, s, Z, L.d_zix, L.d_cols,
                           L.d_views, L.adj, fbase, kappa, out, vg, vper, part);
    LAUNCH_CHECK("k_adj_gather");
    return CBCT_OK;
}

}  // namespace

cbct_status cbct_launch_adjoint(const Level &L, const float *proj, const float *fbase, float kappa, float *out,
                                float *Zws, hipStream_t s, bool preweighted, float *out2) {
    // out2: the view-group sum writes it too; the other paths copy out into it
    const auto copy_out2 = [&]() -> cbct_status {
        if (out2) {
            hipError_t e = hipMemcpyAsync(out2, out, sizeof(float) * L.nvox(), hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return cbct_hip_error(e, "adjoint: copy of the result");
        }
        return CBCT_OK;
    };
    size_t lds = sizeof(double2) * (L.nv + 1 + L.zk_max);
    const bool gb_lds = lds <= 64 * 1024;
    if (!gb_lds) lds = sizeof(double2) * (L.nv + 1);
    dim3 g1(L.nu, L.nviews);
    // columns of more than 256 rows take 512 threads: their prefix sums in one pass (P^T at
    // 512x512x64 / 40 views, 384 rows, 1.47-1.49 against 1.51 ms; at 192 rows 512 threads took
    // 0.268 against 0.260 ms).  The sums, and so the profiles, do not depend on the block size.
    const int pb = L.nv > 256 ? 512 : 256;
    if (preweighted)
        hipLaunchKernelGGL((k_adj_profiles<true>), g1, dim3(pb), lds, s, proj, L.d_cols, L.d_zix, L.nu, L.nv, L.nz,
                           (float)L.pv, gb_lds, Zws);
    else
        hipLaunchKernelGGL((k_adj_profiles<false>), g1, dim3(pb), lds, s, proj, L.d_cols, L.d_zix, L.nu, L.nv, L.nz,
                           (float)L.pv, gb_lds, Zws);
    LAUNCH_CHECK("k_adj_profiles");
    const int nz = L.nz;
    const int tzs = cbct_adj_staged_tz(nz);  // 32 or 0
    cbct_status st;
    if (tzs) {
        const int vg = L.adj_vsplit, vper = (L.nviews + vg - 1) / vg;
        float *part = Zws + L.adj_part_off;
        dim3 grid((L.nx + ADJ_TX - 1) / ADJ_TX, (L.ny + ADJ_TY - 1) / ADJ_TY, (nz / tzs) * vg);
        hipLaunchKernelGGL((k_adj_gather_staged<32, GS_ROWS32>), grid, dim3(ADJ_TX * ADJ_TY), 0, s, Zws, L.d_zix,
                           L.d_cols, L.d_views, L.adj, vg, vper, fbase, kappa, out, out2, part);
        LAUNCH_CHECK("k_adj_gather_staged");
        if (vg > 1) {
            const long n = L.nvox();
            const int nb = (int)std::min<long>((n + 255) / 256, 4096);
            hipLaunchKernelGGL(k_adj_combine, dim3(nb), dim3(256), 0, s, part, vg, n, fbase, kappa, out, out2);
            LAUNCH_CHECK("k_adj_combine");
        }
        return CBCT_OK;  // one view group: the gather wrote out2
    }
    // other depths: per-lane gather, z cells per thread up to 64 (the window and weight work per
    // voxel column and view is shared by all its cells), views split into groups on small grids
    const int vg = L.adj_vsplit, vper = (L.nviews + vg - 1) / vg;
    float *part = Zws + L.adj_part_off;
    switch (cbct_adj_lane_tz(nz)) {
        case 64: st = launch_gather<64>(L, Zws, fbase, kappa, out, vg, vper, part, s); break;
        case 32: st = launch_gather<32>(L, Zws, fbase, kappa, out, vg, vper, part, s); break;
        case 16: st = launch_gather<16>(L, Zws, fbase, kappa, out, vg, vper, part, s); break;
        default: st = launch_gather<8>(L, Zws, fbase, kappa, out, vg, vper, part, s); break;
    }
    if (st) return st;
    if (vg > 1) {
        const long n = L.nvox();
        const int nb = (int)std::min<long>((n + 255) / 256, 4096);
        hipLaunchKernelGGL(k_adj_combine, dim3(nb), dim3(256), 0, s, part, vg, n, fbase, kappa, out, out2);
        LAUNCH_CHECK("k_adj_combine");
        return CBCT_OK;
    }
    return copy_out2();
}

cbct_status cbct_launch_adjoint_batch(const AdjReq *r, int n, hipStream_t s, int *launches, int *items) {
    int nl = 0, ni = 0;
    cbct_status st;
    std::vector<int> staged;
    for (int q = 0; q < n; q++) {
        if (cbct_adj_staged_tz(r[q].L->nz)) {
            staged.push_back(q);
            continue;
        }
        // the per-lane gather: a solo launch sequence
        if ((st = cbct_launch_adjoint(*r[q].L, r[q].proj, r[q].fbase, r[q].kappa, r[q].out, r[q].Zws, s, true,
                                      r[q].out2)))
            return st;
        nl += 3;
        ni += 3;
    }
    for (size_t q0 = 0; q0 < staged.size(); q0 += CBCT_MAXB) {
        const int m = (int)std::min<size_t>(CBCT_MAXB, staged.size() - q0);
        BPr P{};
        BGa G{};
        BCo C{};
        size_t lds = 0;
        int wp = 0, wg = 0, wc = 0;
        for (int j = 0; j < m; j++) {
            const AdjReq &a = r[staged[q0 + j]];
            const Level &L = *a.L;
            // the same LDS table choice as a solo launch
            size_t l1 = sizeof(double2) * (L.nv + 1 + L.zk_max);
            const bool gb = l1 <= 64 * 1024;
            if (!gb) l1 = sizeof(double2) * (L.nv + 1);
            lds = std::max(lds, l1);
            P.it[j] = BPrItem{a.proj, L.d_cols, L.d_zix, a.Zws, L.nu, L.nv, L.nz, L.nviews, gb ? 1 : 0, (float)L.pv};
            P.wg0[j] = wp;
            wp += cbct_batch_pad(L.nu * L.nviews);
            const int vg = L.adj_vsplit, vper = (L.nviews + vg - 1) / vg;
            const int ntx = (L.nx + ADJ_TX - 1) / ADJ_TX, nty = (L.ny + ADJ_TY - 1) / ADJ_TY;
            float *part = a.Zws + L.adj_part_off;
            G.it[j] = BGaItem{a.Zws, L.d_zix, L.d_cols, L.d_views, a.fbase, a.out, a.out2, part, L.adj,
                              ntx, nty, vg, vper, a.kappa};
            G.wg0[j] = wg;
            wg += cbct_batch_pad(ntx * nty * (L.nz / 32) * vg);
            if (vg > 1) {
                const long nvox = L.nvox();
                C.it[C.n] = BCoItem{part, a.fbase, a.out, a.out2, nvox, vg, a.kappa};
                C.wg0[C.n] = wc;
                wc += (int)std::min<long>((nvox + 255) / 256, 4096);
                C.n++;
            }
        }
        P.n = G.n = m;
        P.wg0[m] = wp;
        G.wg0[m] = wg;
        C.wg0[C.n] = wc;
        hipLaunchKernelGGL(k_adj_profiles_b, dim3(wp), dim3(256), lds, s, P);
        LAUNCH_CHECK("k_adj_profiles_b");
        hipLaunchKernelGGL(k_adj_gather_staged_b, dim3(wg), dim3(ADJ_TX * ADJ_TY), 0, s, G);
        LAUNCH_CHECK("k_adj_gather_staged_b");
        nl += 2;
        ni += 2 * m;
        if (C.n) {
            hipLaunchKernelGGL(k_adj_combine_b, dim3(wc), dim3(256), 0, s, C);
            LAUNCH_CHECK("k_adj_combine_b");
            nl++;
            ni += C.n;
        }
    }
    if (launches) *launches = nl;
    if (items) *items = ni;
    return CBCT_OK;
}
