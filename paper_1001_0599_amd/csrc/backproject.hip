// Adjoint P^T: the exact transpose of the forward projector, as a voxel-driven gather with
// no atomics (Section II.C.2 of the paper explains why a ray-driven scatter is a poor fit for
// GPUs: threads collide on voxels).
//
// P sums, for every ray (view t, column i, row j) and sample k, w_ij * Lx Ly Lz f, where Lx Ly
// are the bilinear weights of the sample's transverse position (shared by all rows of the
// column) and Lz the linear weight of the row's z index s_kj = gamma_k q_j + (nz-1)/2.  Hence
//   (P^T y)_abc = sum_t sum_i sum_k Lx(a) Ly(b) Z_tik(c),  Z_tik(c) = sum_j w_ij y_tji hat(s_kj - c).
// One work-group owns a tile of 16 x 16 voxel columns and TZ z cells and keeps its sums in
// registers across all views.  Per view and per group of 8 detector columns crossing the tile:
//   1. FP64 prefix sums A[J] = sum_{J'<J} W_J', B[J] = sum_{J'<J} J' W_J' (W = w y) over the
//      detector rows that can reach the tile (local row index J);
//   2. one slot per (column, sample) whose transverse position lies within one voxel of the
//      tile;
//   3. Z of every slot at the tile's TZ cells, each in O(1) from A and B: the rows with s in
//      [c-1, c) and [c, c+1) are the index ranges [J(c-1), J(c)) and [J(c), J(c+1)) with
//      J(x) = ceil((x - sigma)/gamma), and the hat weights are linear in J on each range;
//   4. each voxel column gathers w = Lx Ly times the slot's Z over its few nearby slots.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "cbct_internal.h"

namespace {

// index of the first local row with s >= x (rows J in [0, nr) have s = gamma J + sigma)
__device__ __forceinline__ int row_bound(float x, float sigma, float inv_gamma, int nr) {
    const float t = ceilf((x - sigma) * inv_gamma);
    return (int)fminf(fmaxf(t, 0.0f), (float)nr);
}

__device__ __forceinline__ void project_uv(float x, float y, float z, float cs, float sn, float sad, float sdd,
                                           float &u, float &v) {
    const float d = fmaf(x, cs, fmaf(y, sn, sad));
    const float inv = sdd / d;
    u = fmaf(x, sn, -y * cs) * inv;
    v = z * inv;
}

template <int TZ>
__global__ void __launch_bounds__(256)
    k_adjoint(const float *__restrict__ proj, const ColParams *__restrict__ cols, const ViewParams *__restrict__ views,
              int nx, int ny, int nz, int nu, int nv, int nviews, float hx, float hy, float hz, float pu, float pv,
              float sad, float sdd, int maxnk, const float *__restrict__ fbase, float kappa,
              float *__restrict__ out) {
    constexpr int ZS = TZ + 4;  // Z row stride (floats), keeps float4 alignment
    extern __shared__ double ldsd[];
    double2 *AB = reinterpret_cast<double2 *>(ldsd);                   // [ADJ_CC][ADJ_MAXR + 1]
    float *Z = reinterpret_cast<float *>(AB + ADJ_CC * (ADJ_MAXR + 1));  // [ADJ_CC * maxnk][ZS]
    __shared__ int s_k0[ADJ_CC], s_n[ADJ_CC], s_base[ADJ_CC + 1];

    const int tid = threadIdx.x;
    const int ta = tid % ADJ_TX, tb = tid / ADJ_TX;
    const int a0 = blockIdx.x * ADJ_TX, b0 = blockIdx.y * ADJ_TY, c0 = blockIdx.z * TZ;
    const int a1 = min(a0 + ADJ_TX, nx) - 1, b1 = min(b0 + ADJ_TY, ny) - 1, c1 = min(c0 + TZ, nz) - 1;
    const int a = a0 + ta, b = b0 + tb;
    const float cx = 0.5f * (float)(nx - 1), cy = 0.5f * (float)(ny - 1), cz = 0.5f * (float)(nz - 1);
    // tile support (voxel centres +- one voxel), mm
    const float xlo = ((float)(a0 - 1) - cx) * hx, xhi = ((float)(a1 + 1) - cx) * hx;
    const float ylo = ((float)(b0 - 1) - cy) * hy, yhi = ((float)(b1 + 1) - cy) * hy;
    const float zlo = ((float)(c0 - 1) - cz) * hz, zhi = ((float)(c1 + 1) - cz) * hz;
    // own support
    const float vx = ((float)a - cx) * hx, vy = ((float)b - cy) * hy;

    float acc[TZ];
#pragma unroll
    for (int q = 0; q < TZ; q++) acc[q] = 0.0f;

    const int wave = tid >> 6, lane = tid & 63;

    for (int view = 0; view < nviews; view++) {
        const ViewParams vp = views[view];
        float umin = FLT_MAX, umax = -FLT_MAX, vmin = FLT_MAX, vmax = -FLT_MAX;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            float u, v;
            project_uv((q & 1) ? xhi : xlo, (q & 2) ? yhi : ylo, (q & 4) ? zhi : zlo, vp.cs, vp.sn, sad, sdd, u, v);
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
            vmin = fminf(vmin, v);
            vmax = fmaxf(vmax, v);
        }
        const float iu = 0.5f * (float)(nu - 1), iv = 0.5f * (float)(nv - 1);
        const int i0 = max(0, (int)floorf(umin / pu + iu) - 1), i1 = min(nu - 1, (int)ceilf(umax / pu + iu) + 1);
        const int j0 = max(0, (int)floorf(vmin / pv + iv) - 1), j1 = min(nv - 1, (int)ceilf(vmax / pv + iv) + 1);
        if (i0 > i1 || j0 > j1) continue;
        // this voxel column's detector columns
        float oumin = FLT_MAX, oumax = -FLT_MAX;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            float u, v;
            project_uv(vx + ((q & 1) ? hx : -hx), vy + ((q & 2) ? hy : -hy), 0.0f, vp.cs, vp.sn, sad, sdd, u, v);
            oumin = fminf(oumin, u);
            oumax = fmaxf(oumax, u);
        }
        const int oi0 = (int)floorf(oumin / pu + iu) - 1, oi1 = (int)ceilf(oumax / pu + iu) + 1;

        for (int ci0 = i0; ci0 <= i1; ci0 += ADJ_CC) {
            const int ncol = min(ADJ_CC, i1 - ci0 + 1);
            __syncthreads();  // previous group's gather is done with Z and the slot tables
            if (tid < ncol) {
                const ColParams cp = cols[(long)view * nu + ci0 + tid];
                // samples with fx in (a0-1, a1+1) and fy in (b0-1, b1+1), widened by one
                float lo = (float)cp.klo, hi = (float)cp.khi;
                if (fabsf(cp.dfx) > 1e-12f) {
                    const float ka = ((float)(a0 - 1) - cp.fx0) / cp.dfx, kb = ((float)(a1 + 1) - cp.fx0) / cp.dfx;
                    lo = fmaxf(lo, fminf(ka, kb) - 1.0f);
                    hi = fminf(hi, fmaxf(ka, kb) + 1.0f);
                }
                if (fabsf(cp.dfy) > 1e-12f) {
                    const float ka = ((float)(b0 - 1) - cp.fy0) / cp.dfy, kb = ((float)(b1 + 1) - cp.fy0) / cp.dfy;
                    lo = fmaxf(lo, fminf(ka, kb) - 1.0f);
                    hi = fminf(hi, fmaxf(ka, kb) + 1.0f);
                }
                const int klo = (int)ceilf(lo), khi = (int)floorf(hi);
                s_k0[tid] = klo;
                s_n[tid] = min(max(khi - klo + 1, 0), maxnk);
            }
            __syncthreads();
            if (tid == 0) {
                int sacc = 0;
                for (int t = 0; t < ncol; t++) {
                    s_base[t] = sacc;
                    sacc += s_n[t];
                }
                s_base[ncol] = sacc;
            }
            __syncthreads();
            const int nslots = s_base[ncol];

            for (int rj0 = j0; rj0 <= j1; rj0 += ADJ_MAXR) {
                const int nr = min(ADJ_MAXR, j1 - rj0 + 1);
                if (rj0 != j0) __syncthreads();  // previous row group's Z pass is done with AB
                // 1. prefix sums, one wave per column
                for (int t = wave; t < ncol; t += 4) {
                    const int col = ci0 + t;
                    const ColParams cp = cols[(long)view * nu + col];
                    double carry_a = 0.0, carry_b = 0.0;
                    double2 *ab = AB + t * (ADJ_MAXR + 1);
                    if (lane == 0) ab[0] = make_double2(0.0, 0.0);
                    for (int r = 0; r < nr; r += 64) {
                        const int J = r + lane;
                        double wv = 0.0;
                        if (J < nr) {
                            const int j = rj0 + J;
                            const float v = ((float)j - iv) * pv;
                            const float w = cp.wsc * sqrtf(fmaf(v, v, cp.r2));
                            wv = (double)(w * proj[((long)view * nv + j) * nu + col]);
                        }
                        double sa = wv, sb = wv * (double)J;
#pragma unroll
                        for (int o = 1; o < 64; o <<= 1) {
                            const double ta_ = __shfl_up(sa, o), tb_ = __shfl_up(sb, o);
                            if (lane >= o) {
                                sa += ta_;
                                sb += tb_;
                            }
                        }
                        if (J < nr) ab[J + 1] = make_double2(carry_a + sa, carry_b + sb);
                        carry_a += __shfl(sa, 63);
                        carry_b += __shfl(sb, 63);
                    }
                }
                __syncthreads();
                // 3. Z of each slot at the tile's cells
                for (int sl = tid; sl < nslots; sl += blockDim.x) {
                    int t = 0;
                    while (t + 1 < ncol && s_base[t + 1] <= sl) t++;
                    const int k = s_k0[t] + (sl - s_base[t]);
                    const ColParams cp = cols[(long)view * nu + ci0 + t];
                    const float gamma = fmaf((float)k, cp.dg, cp.g0);
                    const float inv_g = 1.0f / gamma;
                    const float sigma = fmaf(gamma, (float)rj0 - iv, cz);
                    const double gd = (double)gamma, sd = (double)sigma;
                    const double2 *ab = AB + t * (ADJ_MAXR + 1);
                    int jp = row_bound((float)(c0 - 1), sigma, inv_g, nr);
                    int jc = row_bound((float)c0, sigma, inv_g, nr);
                    double2 Ap = ab[jp], Ac = ab[jc];
                    float *zrow = Z + sl * ZS;
#pragma unroll
                    for (int q = 0; q < TZ; q++) {
                        const int c = c0 + q;
                        const int jn = row_bound((float)(c + 1), sigma, inv_g, nr);
                        const double2 An = ab[jn];
                        const double dal = Ac.x - Ap.x, dbl = Ac.y - Ap.y;  // rows with s in [c-1, c)
                        const double dah = An.x - Ac.x, dbh = An.y - Ac.y;  // rows with s in [c, c+1)
                        const double cc = (double)c;
                        const double zc = gd * (dbl - dbh) + (sd - cc + 1.0) * dal + (cc + 1.0 - sd) * dah;
                        if (rj0 == j0)
                            zrow[q] = (float)zc;
                        else
                            zrow[q] += (float)zc;
                        Ap = Ac;
                        Ac = An;
                    }
                }
            }
            __syncthreads();
            // 4. gather over this voxel column's slots
            const int g0 = max(oi0, ci0), g1 = min(oi1, ci0 + ncol - 1);
            for (int col = g0; col <= g1; col++) {
                const int t = col - ci0;
                const ColParams cp = cols[(long)view * nu + col];
                float lo = (float)s_k0[t], hi = (float)(s_k0[t] + s_n[t] - 1);
                if (fabsf(cp.dfx) > 1e-12f) {
                    const float ka = ((float)(a - 1) - cp.fx0) / cp.dfx, kb = ((float)(a + 1) - cp.fx0) / cp.dfx;
                    lo = fmaxf(lo, fminf(ka, kb) - 1.0f);
                    hi = fminf(hi, fmaxf(ka, kb) + 1.0f);
                }
                if (fabsf(cp.dfy) > 1e-12f) {
                    const float ka = ((float)(b - 1) - cp.fy0) / cp.dfy, kb = ((float)(b + 1) - cp.fy0) / cp.dfy;
                    lo = fmaxf(lo, fminf(ka, kb) - 1.0f);
                    hi = fminf(hi, fmaxf(ka, kb) + 1.0f);
                }
                const int klo = (int)ceilf(lo), khi = (int)floorf(hi);
                for (int k = klo; k <= khi; k++) {
                    const float kf = (float)k;
                    const float fx = fmaf(kf, cp.dfx, cp.fx0), fy = fmaf(kf, cp.dfy, cp.fy0);
                    const float wxy = fmaxf(1.0f - fabsf(fx - (float)a), 0.0f) * fmaxf(1.0f - fabsf(fy - (float)b), 0.0f);
                    if (wxy == 0.0f) continue;
                    const float4 *zr = reinterpret_cast<const float4 *>(Z + (s_base[t] + k - s_k0[t]) * ZS);
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
    if (a < nx && b < ny) {
#pragma unroll
        for (int q = 0; q < TZ; q++) {
            const int c = c0 + q;
            if (c < nz) {
                const long idx = ((long)c * ny + b) * nx + a;
                out[idx] = fbase ? fmaf(-kappa, acc[q], fbase[idx]) : acc[q];
            }
        }
    }
}

template <int TZ>
cbct_status launch_adj(const Level &L, const float *proj, const float *fbase, float kappa, float *out, hipStream_t s) {
    const size_t lds = sizeof(double2) * ADJ_CC * (ADJ_MAXR + 1) + sizeof(float) * ADJ_CC * L.adj_maxnk * (TZ + 4);
    dim3 grid((L.nx + ADJ_TX - 1) / ADJ_TX, (L.ny + ADJ_TY - 1) / ADJ_TY, (L.nz + TZ - 1) / TZ);
    hipLaunchKernelGGL((k_adjoint<TZ>), grid, dim3(ADJ_TX * ADJ_TY), lds, s, proj, L.d_cols, L.d_views, L.nx, L.ny,
                       L.nz, L.nu, L.nv, L.nviews, (float)L.hx, (float)L.hy, (float)L.hz, (float)L.pu, (float)L.pv,
                       (float)L.sad, (float)L.sdd, L.adj_maxnk, fbase, kappa, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_adjoint launch");
    return CBCT_OK;
}

}  // namespace

cbct_status cbct_launch_adjoint(const Level &L, const float *proj, const float *fbase, float kappa, float *out,
                                hipStream_t s) {
    if (L.adj_tz == 16) return launch_adj<16>(L, proj, fbase, kappa, out, s);
    return launch_adj<8>(L, proj, fbase, kappa, out, s);
}
