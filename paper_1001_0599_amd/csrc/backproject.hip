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
//  2. gather: a work-group owns 16 x 16 voxel columns and 16 (or 8) z cells and keeps its sums
//     in registers across all views; per view each voxel column visits the detector columns and
//     samples whose bilinear footprint covers it (exact windows) and adds Lx Ly times the
//     sample's profile segment (float4 loads, shared through the caches by neighbouring voxels).
#include <hip/hip_runtime.h>

#include <cfloat>

#include "cbct_internal.h"

namespace {

// ---------------------------------------------------------------------------- pass 1
// PREWEIGHTED: the input already holds w_ij * y (the solver's residual epilogue writes it)
template <bool PREWEIGHTED>
__global__ void __launch_bounds__(256)
    k_adj_profiles(const float *__restrict__ proj, const ColParams *__restrict__ cols,
                   const ZIndex *__restrict__ zix, int nu, int nv, int nz, float pv, float *__restrict__ Z) {
    extern __shared__ double2 ab[];  // [nv + 1]: (A, B)
    __shared__ double wtot[4][2];
    const int i = blockIdx.x, view = blockIdx.y;
    const long col = (long)view * nu + i;
    const ColParams cp = cols[col];
    const ZIndex zi = zix[col];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float iv = 0.5f * (float)(nv - 1);
    // prefix sums: rows in chunks of 256, each chunk scanned by the block (wave scans + wave totals)
    double carry_a = 0.0, carry_b = 0.0;
    if (tid == 0) ab[0] = make_double2(0.0, 0.0);
    for (int j0 = 0; j0 < nv; j0 += 256) {
        const int j = j0 + tid;
        double wa = 0.0, wb = 0.0;
        if (j < nv) {
            float w = proj[((long)view * nv + j) * nu + i];
            const float q = (float)j - iv;
            if (!PREWEIGHTED) {
                const float v = q * pv;
                w *= cp.wsc * sqrtf(fmaf(v, v, cp.r2));
            }
            wa = (double)w;
            wb = (double)w * (double)q;
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
        for (int w = 0; w < 4; w++) {
            carry_a += wtot[w][0];
            carry_b += wtot[w][1];
        }
        __syncthreads();
    }
    // profiles: items (sample, 4 consecutive cells), cells fastest
    const double beta = 0.5 * (double)(nz - 1);
    const int nq = (nz + 3) >> 2;
    float *zc = Z + zi.off;
    for (int it = tid; it < zi.nk * nq; it += blockDim.x) {
        const int kk = it / nq, c4 = (it - kk * nq) << 2;
        const double gamma = (double)fmaf((float)(zi.k0 + kk), cp.dg, cp.g0);
        const double ig = 1.0 / gamma;
        int jb[6];
#pragma unroll
        for (int q = 0; q < 6; q++) {
            const double x = (double)(c4 - 1 + q);
            const double r = ceil((x - beta) * ig + (double)iv);
            jb[q] = (int)fmin(fmax(r, 0.0), (double)nv);
        }
        double2 pr[6];
#pragma unroll
        for (int q = 0; q < 6; q++) pr[q] = ab[jb[q]];
        float out[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const double c = (double)(c4 + q);
            const double dal = pr[q + 1].x - pr[q].x, dbl = pr[q + 1].y - pr[q].y;          // s in [c-1, c)
            const double dah = pr[q + 2].x - pr[q + 1].x, dbh = pr[q + 2].y - pr[q + 1].y;  // s in [c, c+1)
            out[q] = (float)(gamma * (dbl - dbh) + (beta - c + 1.0) * dal + (c + 1.0 - beta) * dah);
        }
        float *dst = zc + (long)kk * nz + c4;
        if ((nz & 3) == 0) {
            *reinterpret_cast<float4 *>(dst) = make_float4(out[0], out[1], out[2], out[3]);
        } else {
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (c4 + q < nz) dst[q] = out[q];
        }
    }
}

// ---------------------------------------------------------------------------- pass 2
// samples k of a column whose index coordinates lie in the open box (xa, xb) x (ya, yb),
// intersected with [lo, hi]; the caller takes klo = floor(lo) + 1, khi = ceil(hi) - 1.  A sample
// on the box boundary has interpolation weight 0 for the voxels inside.
__device__ __forceinline__ void sample_window(const ColParams &cp, float xa, float xb, float ya, float yb, float &lo,
                                              float &hi) {
    if (cp.idfx != 0.0f) {
        const float ka = (xa - cp.fx0) * cp.idfx, kb = (xb - cp.fx0) * cp.idfx;
        lo = fmaxf(lo, fminf(ka, kb));
        hi = fminf(hi, fmaxf(ka, kb));
    }
    if (cp.idfy != 0.0f) {
        const float ka = (ya - cp.fy0) * cp.idfy, kb = (yb - cp.fy0) * cp.idfy;
        lo = fmaxf(lo, fminf(ka, kb));
        hi = fminf(hi, fmaxf(ka, kb));
    }
}

template <int TZ, bool VEC>
__global__ void __launch_bounds__(256)
    k_adj_gather(const float *__restrict__ Z, const ZIndex *__restrict__ zix, const ColParams *__restrict__ cols,
                 const ViewParams *__restrict__ views, AdjArgs A, const float *__restrict__ fbase, float kappa,
                 float *__restrict__ out) {
    const int tid = threadIdx.x;
    const int a = blockIdx.x * ADJ_TX + tid % ADJ_TX, b = blockIdx.y * ADJ_TY + tid / ADJ_TX;
    const int c0 = blockIdx.z * TZ;
    const float cx = 0.5f * (float)(A.nx - 1), cy = 0.5f * (float)(A.ny - 1);
    const float iu = 0.5f * (float)(A.nu - 1), ipu = 1.0f / A.pu;
    const float vx = ((float)a - cx) * A.hx, vy = ((float)b - cy) * A.hy;
    if (a >= A.nx || b >= A.ny) return;

    float acc[TZ];
#pragma unroll
    for (int q = 0; q < TZ; q++) acc[q] = 0.0f;

    for (int view = 0; view < A.nviews; view++) {
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
#pragma unroll
    for (int q = 0; q < TZ; q++) {
        const int c = c0 + q;
        if (c < A.nz) {
            const long idx = ((long)c * A.ny + b) * A.nx + a;
            out[idx] = fbase ? fmaf(-kappa, acc[q], fbase[idx]) : acc[q];
        }
    }
}

#define LAUNCH_CHECK(what)                                     \
    do {                                                       \
        hipError_t e_ = hipGetLastError();                     \
        if (e_ != hipSuccess) return cbct_hip_error(e_, what); \
    } while (0)

template <int TZ>
cbct_status launch_gather(const Level &L, const float *Z, const float *fbase, float kappa, float *out, hipStream_t s) {
    dim3 grid((L.nx + ADJ_TX - 1) / ADJ_TX, (L.ny + ADJ_TY - 1) / ADJ_TY, (L.nz + TZ - 1) / TZ);
    if (L.nz % TZ == 0)
        hipLaunchKernelGGL((k_adj_gather<TZ, true>), grid, dim3(ADJ_TX * ADJ_TY), 0, s, Z, L.d_zix, L.d_cols,
                           L.d_views, L.adj, fbase, kappa, out);
    else
        hipLaunchKernelGGL((k_adj_gather<TZ, false>), grid, dim3(ADJ_TX * ADJ_TY), 0, s, Z, L.d_zix, L.d_cols,
                           L.d_views, L.adj, fbase, kappa, out);
    LAUNCH_CHECK("k_adj_gather");
    return CBCT_OK;
}

}  // namespace

cbct_status cbct_launch_adjoint(const Level &L, const float *proj, const float *fbase, float kappa, float *out,
                                float *Zws, hipStream_t s, bool preweighted) {
    const size_t lds = sizeof(double2) * (L.nv + 1);
    dim3 g1(L.nu, L.nviews);
    if (preweighted)
        hipLaunchKernelGGL((k_adj_profiles<true>), g1, dim3(256), lds, s, proj, L.d_cols, L.d_zix, L.nu, L.nv, L.nz,
                           (float)L.pv, Zws);
    else
        hipLaunchKernelGGL((k_adj_profiles<false>), g1, dim3(256), lds, s, proj, L.d_cols, L.d_zix, L.nu, L.nv, L.nz,
                           (float)L.pv, Zws);
    LAUNCH_CHECK("k_adj_profiles");
    if (L.nz >= 16) return launch_gather<16>(L, Zws, fbase, kappa, out, s);
    return launch_gather<8>(L, Zws, fbase, kappa, out, s);
}
