// Adjoint P^T: the exact transpose of the forward projector, as a voxel-driven gather with
// no atomics (Section II.C.2 of the paper explains why a ray-driven scatter is a poor fit for
// GPUs: threads collide on voxels).
//
// P sums, for every ray (view t, column i, row j) and sample k, w_ij * Lx Ly Lz f, where Lx Ly
// are the bilinear weights of the sample's transverse position (shared by all rows of the
// column) and Lz the linear weight of the row's z index s_kj = gamma_k q_j + (nz-1)/2.  Hence
//   (P^T y)_abc = sum_t sum_i sum_k Lx(a) Ly(b) Z_tik(c),  Z_tik(c) = sum_j w_ij y_tji hat(s_kj - c).
// One work-group owns a tile of 16 x 16 voxel columns and TZ z cells and keeps its sums in
// registers across all views.  Per view, the detector columns crossing the tile are processed in
// chunks sized to LDS; per chunk:
//   a. the column parameters are staged in LDS, and one wave assigns a slot to every (column,
//      sample) whose transverse position lies within one voxel of the tile;
//   b. the weighted projections W = w y of the rows that can reach the tile are loaded with
//      coalesced reads;
//   c. prefix sums A[J] = sum_{J'<J} W_J', B[J] = sum_{J'<J} (J' - Jm) W_J' along each column
//      (rows centred on the chunk's middle row Jm to limit cancellation), in 16-row blocks;
//   d. Z of every slot at the tile's TZ cells, each in O(1) from A and B: the rows with s in
//      [c-1, c) and [c, c+1) are the index ranges [J(c-1), J(c)) and [J(c), J(c+1)) with
//      J(x) = ceil((x - sigma)/gamma), and the hat weights are linear in J on each range;
//   e. each voxel column gathers Lx Ly times the slot's Z over its nearby slots.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "cbct_internal.h"

namespace {

constexpr int RB = 16;  // rows per prefix-sum block
constexpr int ZH = 8;   // cells per Z work item

// q / n for 0 <= q < 2^20 and 1 <= n <= 64, via a float reciprocal with one correction step
__device__ __forceinline__ void divmod_small(int q, int n, float inv_n, int &d, int &r) {
    d = (int)((float)q * inv_n);
    r = q - d * n;
    if (r >= n) { d++; r -= n; }
    if (r < 0) { d--; r += n; }
}

// samples k of a column whose index coordinates lie in (xa, xb) x (ya, yb), widened by one,
// intersected with [lo, hi]
__device__ __forceinline__ void sample_window(float fx0, float fy0, float idfx, float idfy, float xa, float xb,
                                              float ya, float yb, float &lo, float &hi) {
    if (idfx != 0.0f) {
        const float ka = (xa - fx0) * idfx, kb = (xb - fx0) * idfx;
        lo = fmaxf(lo, fminf(ka, kb) - 1.0f);
        hi = fminf(hi, fmaxf(ka, kb) + 1.0f);
    }
    if (idfy != 0.0f) {
        const float ka = (ya - fy0) * idfy, kb = (yb - fy0) * idfy;
        lo = fmaxf(lo, fminf(ka, kb) - 1.0f);
        hi = fminf(hi, fmaxf(ka, kb) + 1.0f);
    }
}

// PREWEIGHTED: the input already holds w_ij * y (the solver's residual epilogue writes it)
template <int TZ, bool PREWEIGHTED>
__global__ void __launch_bounds__(256, 3)
    k_adjoint(const float *__restrict__ proj, const ColParams *__restrict__ cols, const ViewParams *__restrict__ views,
              AdjArgs A, const float *__restrict__ fbase, float kappa, float *__restrict__ out) {
    constexpr int ZS = TZ + 4;  // Z row stride (floats), keeps float4 alignment
    constexpr int NH = TZ / ZH;
    extern __shared__ float4 lds4[];
    const int CC = A.cc_max, RM = A.r_max, NBM = (A.r_max + RB - 1) / RB;
    ColParams *cpl = reinterpret_cast<ColParams *>(lds4);                   // [CC]
    int *sk0 = reinterpret_cast<int *>(cpl + CC);                           // [CC]
    int *sn = sk0 + CC;                                                     // [CC]
    int *sbase = sn + CC;                                                   // [CC + 1]
    int *scol = sbase + ((CC + 1 + 3) & ~3);                                // [s_max] slot -> column
    float2 *btot = reinterpret_cast<float2 *>(scol + ((A.s_max + 3) & ~3));  // [CC][NBM]
    float2 *AB = btot + ((CC * NBM + 1) & ~1);                               // [CC][RM + 1]
    float *Z = reinterpret_cast<float *>(AB + ((CC * (RM + 1) + 1) & ~1));   // [s_max][ZS]
    const int ABS = RM + 1;

    const int tid = threadIdx.x, lane = tid & 63;
    const int ta = tid % ADJ_TX, tb = tid / ADJ_TX;
    const int a0 = blockIdx.x * ADJ_TX, b0 = blockIdx.y * ADJ_TY, c0 = blockIdx.z * TZ;
    const int a1 = min(a0 + ADJ_TX, A.nx) - 1, b1 = min(b0 + ADJ_TY, A.ny) - 1, c1 = min(c0 + TZ, A.nz) - 1;
    const int a = a0 + ta, b = b0 + tb;
    const float cx = 0.5f * (float)(A.nx - 1), cy = 0.5f * (float)(A.ny - 1), cz = 0.5f * (float)(A.nz - 1);
    const float iu = 0.5f * (float)(A.nu - 1), iv = 0.5f * (float)(A.nv - 1);
    const float ipu = 1.0f / A.pu, ipv = 1.0f / A.pv;
    // tile support (voxel centres +- one voxel), mm
    const float xlo = ((float)(a0 - 1) - cx) * A.hx, xhi = ((float)(a1 + 1) - cx) * A.hx;
    const float ylo = ((float)(b0 - 1) - cy) * A.hy, yhi = ((float)(b1 + 1) - cy) * A.hy;
    const float zlo = ((float)(c0 - 1) - cz) * A.hz, zhi = ((float)(c1 + 1) - cz) * A.hz;
    const float vx = ((float)a - cx) * A.hx, vy = ((float)b - cy) * A.hy;

    float acc[TZ];
#pragma unroll
    for (int q = 0; q < TZ; q++) acc[q] = 0.0f;

    for (int view = 0; view < A.nviews; view++) {
        const ViewParams vp = views[view];
        // detector footprint of the tile support: columns [i0, i1], rows [j0, j1]
        float umin = FLT_MAX, umax = -FLT_MAX, vmin = FLT_MAX, vmax = -FLT_MAX;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float x = (q & 1) ? xhi : xlo, y = (q & 2) ? yhi : ylo;
            const float inv = A.sdd * __builtin_amdgcn_rcpf(fmaf(x, vp.cs, fmaf(y, vp.sn, A.sad)));
            const float u = fmaf(x, vp.sn, -y * vp.cs) * inv;
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
            vmin = fminf(vmin, fminf(zlo * inv, zhi * inv));
            vmax = fmaxf(vmax, fmaxf(zlo * inv, zhi * inv));
        }
        const int i0 = max(0, (int)floorf(fmaf(umin, ipu, iu)) - 1);
        const int i1 = min(A.nu - 1, (int)ceilf(fmaf(umax, ipu, iu)) + 1);
        const int j0 = max(0, (int)floorf(fmaf(vmin, ipv, iv)) - 1);
        const int j1 = min(A.nv - 1, (int)ceilf(fmaf(vmax, ipv, iv)) + 1);
        if (i0 > i1 || j0 > j1) continue;  // the tile is outside this view's cone
        // this voxel column's detector columns
        float oumin = FLT_MAX, oumax = -FLT_MAX;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float x = vx + ((q & 1) ? A.hx : -A.hx), y = vy + ((q & 2) ? A.hy : -A.hy);
            const float u = fmaf(x, vp.sn, -y * vp.cs) * A.sdd * __builtin_amdgcn_rcpf(fmaf(x, vp.cs, fmaf(y, vp.sn, A.sad)));
            oumin = fminf(oumin, u);
            oumax = fmaxf(oumax, u);
        }
        const int oi0 = (int)floorf(fmaf(oumin, ipu, iu)) - 1, oi1 = (int)ceilf(fmaf(oumax, ipu, iu)) + 1;

        for (int ci0 = i0; ci0 <= i1; ci0 += CC) {
            const int ncol = min(CC, i1 - ci0 + 1);
            const float inv_ncol = 1.0f / (float)ncol;
            __syncthreads();  // the previous chunk's gather is done with LDS
            // a. column parameters, slots and the slot -> column map (one wave; ncol <= 64)
            if (tid < 64) {
                int n = 0, klo = 0;
                if (lane < ncol) {
                    const ColParams cp = cols[(long)view * A.nu + ci0 + lane];
                    cpl[lane] = cp;
                    float lo = (float)cp.klo, hi = (float)cp.khi;
                    sample_window(cp.fx0, cp.fy0, cp.idfx, cp.idfy, (float)(a0 - 1), (float)(a1 + 1), (float)(b0 - 1),
                                  (float)(b1 + 1), lo, hi);
                    klo = (int)ceilf(lo);
                    n = min(max((int)floorf(hi) - klo + 1, 0), A.maxnk);
                }
                int incl = n;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int t = __shfl_up(incl, o);
                    if (lane >= o) incl += t;
                }
                const int base = incl - n;
                if (lane < ncol) {
                    sk0[lane] = klo;
                    sn[lane] = n;
                    sbase[lane] = base;
                    for (int q = 0; q < n && base + q < A.s_max; q++) scol[base + q] = lane;
                }
                if (lane == ncol - 1) sbase[ncol] = min(incl, A.s_max);
            }
            __syncthreads();
            const int nslots = sbase[ncol];

            for (int rj0 = j0; rj0 <= j1; rj0 += RM) {
                const int nr = min(RM, j1 - rj0 + 1);
                const int nb = (nr + RB - 1) / RB;
                const float rmid = (float)(nr >> 1);
                if (rj0 != j0) __syncthreads();  // the previous row chunk's Z pass is done with AB
                // b. weighted projections of 16-row blocks (loads coalesced along the detector row,
                //    all in flight at once), scanned in registers
                for (int it = tid; it < ncol * nb; it += 256) {
                    int blk, col;
                    divmod_small(it, ncol, inv_ncol, blk, col);
                    const int r0 = blk * RB;
                    const float *src = proj + ((long)view * A.nv + rj0 + r0) * A.nu + ci0 + col;
                    float wr[RB];
#pragma unroll
                    for (int q = 0; q < RB; q++) wr[q] = (r0 + q < nr) ? src[(long)q * A.nu] : 0.0f;
                    if (!PREWEIGHTED) {
                        const float wsc = cpl[col].wsc, r2 = cpl[col].r2;
#pragma unroll
                        for (int q = 0; q < RB; q++) {
                            const float v = ((float)(rj0 + r0 + q) - iv) * A.pv;
                            wr[q] *= wsc * sqrtf(fmaf(v, v, r2));
                        }
                    }
                    float2 *p = AB + col * ABS + r0 + 1;
                    float sa = 0.0f, sbv = 0.0f;
#pragma unroll
                    for (int q = 0; q < RB; q++) {
                        sa += wr[q];
                        sbv = fmaf(wr[q], (float)(r0 + q) - rmid, sbv);
                        if (r0 + q < nr) p[q] = make_float2(sa, sbv);
                    }
                    btot[col * NBM + blk] = make_float2(sa, sbv);
                    if (blk == 0) AB[col * ABS] = make_float2(0.0f, 0.0f);
                }
                __syncthreads();
                // c. add the sums of the preceding blocks
                for (int it = tid; it < ncol * nb; it += 256) {
                    int blk, col;
                    divmod_small(it, ncol, inv_ncol, blk, col);
                    if (blk == 0) continue;
                    float oa = 0.0f, ob = 0.0f;
                    for (int q = 0; q < blk; q++) {
                        const float2 t = btot[col * NBM + q];
                        oa += t.x;
                        ob += t.y;
                    }
                    const int r0 = blk * RB;
                    float2 *p = AB + col * ABS + r0 + 1;
#pragma unroll
                    for (int q = 0; q < RB; q++)
                        if (r0 + q < nr) {
                            const float2 v = p[q];
                            p[q] = make_float2(v.x + oa, v.y + ob);
                        }
                }
                __syncthreads();
                // d. Z of each slot at the tile's cells, ZH cells per work item
                for (int it = tid; it < nslots * NH; it += 256) {
                    const int sl = it / NH, h = it - sl * NH;
                    const int t = scol[sl];
                    const ColParams &cp = cpl[t];
                    const int k = sk0[t] + (sl - sbase[t]);
                    const float gamma = fmaf((float)k, cp.dg, cp.g0);
                    const float inv_g = 1.0f / gamma;
                    // row r of the chunk meets the column's sample at s = gamma (r - rmid) + sigma
                    const float sigma = fmaf(gamma, (float)rj0 + rmid - iv, cz);
                    const float2 *ab = AB + t * ABS;
                    const int cb = c0 + h * ZH;
                    int jb[ZH + 2];
#pragma unroll
                    for (int q = 0; q < ZH + 2; q++) {
                        const float r = ceilf(fmaf((float)(cb - 1 + q) - sigma, inv_g, rmid));
                        jb[q] = (int)fminf(fmaxf(r, 0.0f), (float)nr);
                    }
                    float2 pr[ZH + 2];
#pragma unroll
                    for (int q = 0; q < ZH + 2; q++) pr[q] = ab[jb[q]];
                    float *zrow = Z + sl * ZS + h * ZH;
#pragma unroll
                    for (int q = 0; q < ZH; q++) {
                        const float c = (float)(cb + q);
                        const float dal = pr[q + 1].x - pr[q].x, dbl = pr[q + 1].y - pr[q].y;      // s in [c-1, c)
                        const float dah = pr[q + 2].x - pr[q + 1].x, dbh = pr[q + 2].y - pr[q + 1].y;  // s in [c, c+1)
                        const float zc = fmaf(gamma, dbl - dbh, fmaf(sigma - c + 1.0f, dal, (c + 1.0f - sigma) * dah));
                        zrow[q] = (rj0 == j0) ? zc : zrow[q] + zc;
                    }
                }
            }
            __syncthreads();
            // e. gather over this voxel column's slots
            const int g0 = max(oi0, ci0), g1 = min(oi1, ci0 + ncol - 1);
            for (int col = g0; col <= g1; col++) {
                const int t = col - ci0;
                const float fx0 = cpl[t].fx0, fy0 = cpl[t].fy0, dfx = cpl[t].dfx, dfy = cpl[t].dfy;
                const int k0 = sk0[t], sb0 = sbase[t];
                float lo = (float)k0, hi = (float)(k0 + sn[t] - 1);
                sample_window(fx0, fy0, cpl[t].idfx, cpl[t].idfy, (float)(a - 1), (float)(a + 1), (float)(b - 1),
                              (float)(b + 1), lo, hi);
                const int klo = (int)ceilf(lo), khi = (int)floorf(hi);
                for (int k = klo; k <= khi; k++) {
                    const int sl = sb0 + k - k0;
                    if (sl >= nslots) break;
                    const float kf = (float)k;
                    const float fx = fmaf(kf, dfx, fx0), fy = fmaf(kf, dfy, fy0);
                    const float wxy =
                        fmaxf(1.0f - fabsf(fx - (float)a), 0.0f) * fmaxf(1.0f - fabsf(fy - (float)b), 0.0f);
                    if (wxy == 0.0f) continue;
                    const float4 *zr = reinterpret_cast<const float4 *>(Z + sl * ZS);
#pragma unroll
                    for (int q = 0; q < TZ / 4; q++) {
                        const float4 z4 = zr[q];
                        acc[4 * q + 0] = fmaf(wxy, z4.x, acc[4 * q + 0]);
                        acc[4 * q + 1] = fmaf(wxy, z4.y, acc[4 * q + 1]);
                        acc[4 * q + 2] = fmaf(wxy, z4.z, acc[4 * q + 2]);
                        acc[4 * q + 3] = fmaf(wxy, z4.w, acc[4 * q + 3]);
                    }
                }
            }
        }
    }
    if (a < A.nx && b < A.ny) {
#pragma unroll
        for (int q = 0; q < TZ; q++) {
            const int c = c0 + q;
            if (c < A.nz) {
                const long idx = ((long)c * A.ny + b) * A.nx + a;
                out[idx] = fbase ? fmaf(-kappa, acc[q], fbase[idx]) : acc[q];
            }
        }
    }
}

size_t adj_lds_bytes(const AdjArgs &A, int tz) {
    const int CC = A.cc_max, NBM = (A.r_max + RB - 1) / RB;
    size_t n = sizeof(ColParams) * CC + sizeof(int) * (3 * CC + ((CC + 1 + 3) & ~3) + ((A.s_max + 3) & ~3));
    n = (n + 15) & ~(size_t)15;
    n += sizeof(float2) * (((size_t)CC * NBM + 1) & ~(size_t)1);
    n += sizeof(float2) * (((size_t)CC * (A.r_max + 1) + 1) & ~(size_t)1);
    n += sizeof(float) * (size_t)A.s_max * (tz + 4);
    return n + 64;
}

template <int TZ, bool PW>
cbct_status launch_adj(const Level &L, const float *proj, const float *fbase, float kappa, float *out, hipStream_t s) {
    const size_t lds = adj_lds_bytes(L.adj, TZ);
    dim3 grid((L.nx + ADJ_TX - 1) / ADJ_TX, (L.ny + ADJ_TY - 1) / ADJ_TY, (L.nz + TZ - 1) / TZ);
    hipLaunchKernelGGL((k_adjoint<TZ, PW>), grid, dim3(ADJ_TX * ADJ_TY), lds, s, proj, L.d_cols, L.d_views, L.adj, fbase,
                       kappa, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_adjoint launch");
    return CBCT_OK;
}

}  // namespace

size_t cbct_adjoint_lds_bytes(const AdjArgs &A, int tz) { return adj_lds_bytes(A, tz); }

cbct_status cbct_launch_adjoint(const Level &L, const float *proj, const float *fbase, float kappa, float *out,
                                hipStream_t s, bool preweighted) {
    if (L.adj_tz == 16)
        return preweighted ? launch_adj<16, true>(L, proj, fbase, kappa, out, s)
                           : launch_adj<16, false>(L, proj, fbase, kappa, out, s);
    return preweighted ? launch_adj<8, true>(L, proj, fbase, kappa, out, s)
                       : launch_adj<8, false>(L, proj, fbase, kappa, out, s);
}
