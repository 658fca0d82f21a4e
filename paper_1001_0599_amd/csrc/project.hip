// Forward projection P (Eq. 1 of the paper as a trilinear ray sum) for gfx950.
//
// Column-coherent sampling: the rays of one detector column i share the transverse (xy)
// positions of their samples (the column's transverse line, sample k at transverse distance
// tau_c + k dtau from the source).  So per sample k the bilinear xy interpolation is done once
// for the whole z range ("column values" col_k[c]), and each ray only interpolates col_k
// linearly at its own z index s = gamma_k q_j + (nz-1)/2.
//
// One work-group handles one (view, column).  Per chunk of KC samples:
//   1. the first KC threads compute the four xy corner weights/offsets of each sample;
//   2. all threads build col_k[c] from four z-contiguous voxel columns (volume in the
//      column-major layout [ny][nx][nz], float4 loads) into an LDS table, once in z order (T)
//      and once reversed (R);
//   3. each thread walks the chunk for one mirrored pair of rows (j, nv-1-j): their z indices
//      are s and (nz-1)-s, so one floor/fract serves both rays (T for j, R for the mirror).
// The z range of the tables is zero-padded so that every ray's index stays inside: rays that
// leave the slab read zeros and no clamp is needed in the inner loop.
//
// LDS table layout: row e (z cell incl. padding) holds KC T values then KC R values, row
// stride 2 KC + 1 words: the two reads of a ray step (cells e and e+1) and the two of its
// mirror share one address register with immediate offsets, and the build's writes hit
// distinct banks.
#include <hip/hip_runtime.h>

#include "cbct_internal.h"

namespace {

__global__ void __launch_bounds__(256) k_to_columns(const float *__restrict__ vol, float *__restrict__ vol_t, int nx,
                                                    int ny, int nz) {
    __shared__ float tile[32][33];
    const int b = blockIdx.z;
    const int a0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;
    for (int r = ty; r < 32; r += 8) {
        const int c = c0 + r, a = a0 + tx;
        if (c < nz && a < nx) tile[r][tx] = vol[((long)c * ny + b) * nx + a];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int a = a0 + r, c = c0 + tx;
        if (a < nx && c < nz) vol_t[((long)b * nx + a) * nz + c] = tile[tx][r];
    }
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// KC: samples per chunk (the host pads every column's sample range to whole chunks; the extra
// samples lie outside the grid and contribute zero); NPT: mirrored row pairs per thread;
// VEC: z-contiguous float4 column loads (nz % 4 == 0)
template <int KC, int NPT, bool VEC>
__global__ void __launch_bounds__(256)
    k_forward(const float *__restrict__ vol_t, const ColParams *__restrict__ cols, int nx, int ny, int nz, int nu,
              int nv, float pv, int pad, int tw, const float *__restrict__ ysub, int wres, float *__restrict__ out,
              double *__restrict__ partials) {
    extern __shared__ float lds[];
    constexpr int kc = KC;
    constexpr int S = 2 * KC + 1;
    float *tab = lds;
    float4 *kw = reinterpret_cast<float4 *>(lds + ((tw * S + 3) & ~3));
    int4 *ko = reinterpret_cast<int4 *>(kw + kc);
    __shared__ double wsum[4];

    // adjacent columns of one view sweep nearly the same voxels: keep them on one XCD
    const int w = cbct_xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int i = w % nu, view = w / nu;
    const ColParams cp = cols[(long)view * nu + i];
    const int npairs = (nv + 1) >> 1;
    const int off = pad + 1;

    for (int e = threadIdx.x; e < tw * S; e += blockDim.x) tab[e] = 0.0f;

    float s0[NPT], ds[NPT], acc_t[NPT], acc_r[NPT];
#pragma unroll
    for (int p = 0; p < NPT; p++) {
        const int pp = threadIdx.x + p * blockDim.x;
        const float q = (pp < npairs) ? (float)pp - 0.5f * (float)(nv - 1) : 0.0f;
        s0[p] = fmaf(cp.g0, q, 0.5f * (float)(nz - 1) + (float)off);
        ds[p] = cp.dg * q;
        acc_t[p] = 0.0f;
        acc_r[p] = 0.0f;
    }

    const int nzq = VEC ? (nz >> 2) : nz;
    // this thread's first table item and the per-step advance (block size = dkk * nzq + dcq)
    const int it0_kk = (int)threadIdx.x / nzq, it0_cq = (int)threadIdx.x - it0_kk * nzq;
    const int dkk = (int)blockDim.x / nzq, dcq = (int)blockDim.x - dkk * nzq;
    for (int k0 = cp.klo; k0 <= cp.khi; k0 += KC) {
        constexpr int nk = KC;
        __syncthreads();  // previous chunk's rays are done with the tables
        if (threadIdx.x < nk) {
            const float kf = (float)(k0 + (int)threadIdx.x);
            const float fx = fmaf(kf, cp.dfx, cp.fx0), fy = fmaf(kf, cp.dfy, cp.fy0);
            const float flx = floorf(fx), fly = floorf(fy);
            const float wx = fx - flx, wy = fy - fly;
            const int a = (int)flx, b = (int)fly;
            const bool xa = (a >= 0 && a < nx), xb = (a + 1 >= 0 && a + 1 < nx);
            const bool ya = (b >= 0 && b < ny), yb = (b + 1 >= 0 && b + 1 < ny);
            const int ac0 = min(max(a, 0), nx - 1), ac1 = min(max(a + 1, 0), nx - 1);
            const int bc0 = min(max(b, 0), ny - 1), bc1 = min(max(b + 1, 0), ny - 1);
            kw[threadIdx.x] = make_float4((xa && ya) ? (1.0f - wx) * (1.0f - wy) : 0.0f,
                                          (xb && ya) ? wx * (1.0f - wy) : 0.0f,
                                          (xa && yb) ? (1.0f - wx) * wy : 0.0f, (xb && yb) ? wx * wy : 0.0f);
            ko[threadIdx.x] = make_int4((bc0 * nx + ac0) * nz, (bc0 * nx + ac1) * nz, (bc1 * nx + ac0) * nz,
                                        (bc1 * nx + ac1) * nz);
        }
        __syncthreads();
        // items (sample kk, cell group cq), cq fastest; the item index advances by the block size,
        // so (kk, cq) advance by (dkk, dcq) with one carry (no division per item)
        int ik = it0_kk, iq = it0_cq;
        for (; ik < nk; ik += dkk, iq += dcq) {
            if (iq >= nzq) {
                iq -= nzq;
                ik++;
                if (ik >= nk) break;
            }
            const int kk = ik, cq = iq;
            const float4 w = kw[kk];
            const int4 o = ko[kk];
            if (VEC) {
                const int c = cq << 2;
                const float *vc = vol_t + c;  // column offsets are non-negative: zero-extended adds
                const float4 v0 = *reinterpret_cast<const float4 *>(vc + (unsigned)o.x);
                const float4 v1 = *reinterpret_cast<const float4 *>(vc + (unsigned)o.y);
                const float4 v2 = *reinterpret_cast<const float4 *>(vc + (unsigned)o.z);
                const float4 v3 = *reinterpret_cast<const float4 *>(vc + (unsigned)o.w);
                float col[4];
                col[0] = fmaf(w.w, v3.x, fmaf(w.z, v2.x, fmaf(w.y, v1.x, w.x * v0.x)));
                col[1] = fmaf(w.w, v3.y, fmaf(w.z, v2.y, fmaf(w.y, v1.y, w.x * v0.y)));
                col[2] = fmaf(w.w, v3.z, fmaf(w.z, v2.z, fmaf(w.y, v1.z, w.x * v0.z)));
                col[3] = fmaf(w.w, v3.w, fmaf(w.z, v2.w, fmaf(w.y, v1.w, w.x * v0.w)));
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    tab[(c + u + off) * S + kk] = col[u];
                    tab[(nz - 1 - c - u + off) * S + kc + kk] = col[u];
                }
            } else {
                const int c = cq;
                const float col = fmaf(w.w, vol_t[o.w + c],
                                       fmaf(w.z, vol_t[o.z + c], fmaf(w.y, vol_t[o.y + c], w.x * vol_t[o.x + c])));
                tab[(c + off) * S + kk] = col;
                tab[(nz - 1 - c + off) * S + kc + kk] = col;
            }
        }
        __syncthreads();
        float sb[NPT];
        bool live = false;  // does any of this thread's rays meet the slab within the chunk?
#pragma unroll
        for (int p = 0; p < NPT; p++) {
            sb[p] = fmaf((float)k0, ds[p], s0[p]);
            const float se = fmaf((float)(KC - 1), ds[p], sb[p]);
            live |= fmaxf(sb[p], se) >= (float)(off - 1) && fminf(sb[p], se) < (float)(off + nz);
        }
        // rays outside the slab only read the zero padding: a wave with none inside skips the chunk
        if (!__any(live)) continue;
#pragma unroll
        for (int kk = 0; kk < KC; kk++) {
#pragma unroll
            for (int p = 0; p < NPT; p++) {
                const float s = fmaf((float)kk, ds[p], sb[p]);  // > 0: the tables are padded
                const float fz = __builtin_amdgcn_fractf(s), gz = 1.0f - fz;
                const int e = (int)s;
                const float *t = tab + __mul24(e, S) + kk;
                const float t0 = t[0], t1 = t[S], r0 = t[kc], r1 = t[kc + S];
                acc_t[p] = fmaf(fz, t1, fmaf(gz, t0, acc_t[p]));
                acc_r[p] = fmaf(fz, r1, fmaf(gz, r0, acc_r[p]));
            }
        }
    }

    double part = 0.0;
#pragma unroll
    for (int p = 0; p < NPT; p++) {
        const int pp = threadIdx.x + p * blockDim.x;
        if (pp < npairs) {
            const int j = pp, jm = nv - 1 - pp;
            const float v = ((float)pp - 0.5f * (float)(nv - 1)) * pv;
            const float w = cp.wsc * sqrtf(fmaf(v, v, cp.r2));
            const long o1 = ((long)view * nv + j) * nu + i, o2 = ((long)view * nv + jm) * nu + i;
            float r1 = w * acc_t[p], r2 = w * acc_r[p];
            if (ysub) {
                // residual mode: sum (P f - Y)^2, and hand the adjoint w * (P f - Y) (or P f - Y)
                r1 -= ysub[o1];
                r2 -= ysub[o2];
                part += (double)r1 * (double)r1;
                if (jm != j) part += (double)r2 * (double)r2;
                if (wres) {
                    r1 *= w;
                    r2 *= w;
                }
            }
            out[o1] = r1;
            if (jm != j) out[o2] = r2;
        }
    }
    if (partials) {
        part = wave_sum(part);
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) wsum[wave] = part;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); w++) s += wsum[w];
            partials[(long)view * nu + i] = s;
        }
    }
}

// one float of the volume through a raw buffer resource (byte offset)
__device__ __forceinline__ float ldv(__amdgpu_buffer_rsrc_t r, int off, int, int) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Forward projection by runs.  Within a chunk of KC samples a ray's z index s_k = s_a + k delta
// (k local) stays in one z cell for long stretches (|delta| is a few hundredths of a cell per
// sample), and on such a run the linear interpolation sums in closed form:
//   sum_k [(1 - f_k) col_k[e] + f_k col_k[e+1]],  f_k = (s_a - e) + k delta,
//   = dA_e + (s_a - e)(dA_{e+1} - dA_e) + delta (dK_{e+1} - dK_e),
// with A_e(k) = sum_{k' < k} col_k'[e] and K_e(k) = sum_{k' < k} k' col_k'[e] prefix sums over the
// chunk's samples.  So a ray costs O(runs) = O(chunks + z cells crossed) instead of O(samples).
// Rows j and nv-1-j are mirror images (s' = nz + 1 - s, cell nz - e, fraction 1 - f): they leave
// their cells at the same samples, so one thread sums both from one split computation.
//
// Per chunk: the first KC threads compute the samples' xy corner weights; wave w builds the prefix
// sums of a contiguous slice of the chunk's samples for all z cells (lane = cell, the bilinear
// column values from four z-contiguous voxel columns), the slices are joined by adding the earlier
// slices' totals, and every thread then sums its pair of rays run by run.  The table is cell-major,
// [e][k] with k = 0 .. KC: column e holds voxel e - 1; cells 0 and nz + 1 stay zero, so rays
// leaving the slab read zeros.
__host__ __device__ constexpr size_t runs_lds_bytes_kc(int kc, int nz, int nwaves) {
    // slice totals: one row of nz per builder (a wave, or half a wave for depths of 32 or less)
    return ((size_t)(nz + 2) * (kc + 1) * 8 + 15) / 16 * 16 + (size_t)kc * 32 +
           (size_t)(nz <= 32 ? 2 * nwaves : nwaves) * nz * 8;
}
template <int KC>
__host__ __device__ constexpr size_t runs_lds_bytes(int nz, int nwaves) {
    return runs_lds_bytes_kc(KC, nz, nwaves);
}

template <int KC, int NPT>
__device__ __forceinline__ void forward_runs_body(const float *__restrict__ vol_t, const ColParams *__restrict__ cols,
                                                  int nx, int ny, int nz, int nu, int nv, float pv,
                                                  const float *__restrict__ ysub, int wres, float *__restrict__ out,
                                                  double *__restrict__ partials, int i, int view) {
    static_assert(KC % 8 == 0 && KC >= 8 && KC <= 64, "chunks are whole groups of 8 samples, at most 64");
    extern __shared__ float4 lds4[];
    constexpr int S = KC + 1;  // entries per cell: (A, K) before local sample k = 0 .. KC
    const int tw = nz + 2;
    float2 *tab = reinterpret_cast<float2 *>(lds4);
    float4 *kw = lds4 + ((size_t)tw * S * 8 + 15) / 16;
    int4 *ko = reinterpret_cast<int4 *>(kw + KC);
    float2 *tot = reinterpret_cast<float2 *>(ko + KC);  // [wave][nz]: slice totals
    __shared__ double wsum[4];

    const ColParams cp = cols[(long)view * nu + i];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;

    // k = 0 and the two zero cells are never written again
    for (int e = tid; e < tw; e += nthr) tab[e * S] = make_float2(0.0f, 0.0f);
    for (int k = 1 + tid; k <= KC; k += nthr) {
        tab[k] = make_float2(0.0f, 0.0f);
        tab[(tw - 1) * S + k] = make_float2(0.0f, 0.0f);
    }

    // pair p: rays j = tid + p * nthr (q <= 0) and its mirror nv - 1 - j.  Ray j's z index (table
    // units, voxel c at s = c + 1) is s_k = s0 + k delta; a run in cell e ends at the first sample
    // past the boundary ahead, e + bo: k = ceil((e + bo - s_a) / delta) (a sample exactly on the
    // boundary may go to either cell: the interpolant is continuous there).
    const int npairs = (nv + 1) >> 1;
    float s0[NPT], dl[NPT], idl[NPT], bo[NPT], acc[NPT], accm[NPT];
#pragma unroll
    for (int p = 0; p < NPT; p++) {
        const int j = tid + p * nthr;
        const float q = (j < npairs) ? (float)j - 0.5f * (float)(nv - 1) : 0.0f;
        s0[p] = fmaf(cp.g0, q, 0.5f * (float)(nz - 1) + 1.0f);
        dl[p] = cp.dg * q;
        idl[p] = dl[p] != 0.0f ? 1.0f / dl[p] : 1e30f;
        bo[p] = dl[p] >= 0.0f ? 1.0f : 0.0f;
        acc[p] = 0.0f;
        accm[p] = 0.0f;
    }
    // voxel loads through a raw buffer: 32-bit byte offsets, one add each
    const __amdgpu_buffer_rsrc_t vrs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(vol_t), 0, nx * ny * nz * 4, 0x00020000);
    // the build maps lanes to z cells; at depths of 32 or less each wave's halves take different
    // slices of samples (builder vw, lane vl), so that no lane idles
    const int half = nz <= 32 ? 1 : 0;
    const int vw = half ? 2 * wave + (lane >> 5) : wave, vl = half ? (lane & 31) : lane;
    const int nvw = half ? 2 * nw : nw, lstep = half ? 32 : 64;
    const int sc = ((KC + nvw - 1) / nvw + 7) & ~7;  // slices of whole groups of 8 samples
    const int ka = min(vw * sc, KC), kb = min(ka + sc, KC);

    for (int k0 = cp.klo; k0 <= cp.khi; k0 += KC) {
        __syncthreads();  // the previous chunk's rays are done with the tables
        if (tid < KC) {
            const float kf = (float)(k0 + tid);
            const float fx = fmaf(kf, cp.dfx, cp.fx0), fy = fmaf(kf, cp.dfy, cp.fy0);
            const float flx = floorf(fx), fly = floorf(fy);
            const float wx = fx - flx, wy = fy - fly;
            const int a = (int)flx, b = (int)fly;
            const bool xa = (a >= 0 && a < nx), xb = (a + 1 >= 0 && a + 1 < nx);
            const bool ya = (b >= 0 && b < ny), yb = (b + 1 >= 0 && b + 1 < ny);
            const int ac0 = min(max(a, 0), nx - 1), ac1 = min(max(a + 1, 0), nx - 1);
            const int bc0 = min(max(b, 0), ny - 1), bc1 = min(max(b + 1, 0), ny - 1);
            kw[tid] = make_float4((xa && ya) ? (1.0f - wx) * (1.0f - wy) : 0.0f, (xb && ya) ? wx * (1.0f - wy) : 0.0f,
                                  (xa && yb) ? (1.0f - wx) * wy : 0.0f, (xb && yb) ? wx * wy : 0.0f);
            ko[tid] = make_int4((bc0 * nx + ac0) * nz * 4, (bc0 * nx + ac1) * nz * 4, (bc1 * nx + ac0) * nz * 4,
                                (bc1 * nx + ac1) * nz * 4);  // byte offsets
        }
        __syncthreads();
        // prefix sums of this wave's slice of samples, lane = z cell; groups of RB samples read
        // their weights first and keep all their voxel loads in flight together
        constexpr int RB = 8;
        for (int c = vl; c < nz; c += lstep) {
            float A = 0.0f, K = 0.0f;
            float2 *row = tab + (c + 1) * S + 1;  // entry k + 1 holds the sums over samples < k + 1
            const int c4 = c * 4;
            for (int kk = ka; kk < kb; kk += RB) {
                float4 wq[RB];
                int4 o[RB];
#pragma unroll
                for (int u = 0; u < RB; u++) {
                    wq[u] = kw[kk + u];
                    o[u] = ko[kk + u];
                }
                float v[RB][4];
#pragma unroll
                for (int u = 0; u < RB; u++) {
                    v[u][0] = ldv(vrs, o[u].x + c4, 0, 0);
                    v[u][1] = ldv(vrs, o[u].y + c4, 0, 0);
                    v[u][2] = ldv(vrs, o[u].z + c4, 0, 0);
                    v[u][3] = ldv(vrs, o[u].w + c4, 0, 0);
                }
                const float kf = (float)kk;
#pragma unroll
                for (int u = 0; u < RB; u++) {
                    const float col =
                        fmaf(wq[u].w, v[u][3], fmaf(wq[u].z, v[u][2], fmaf(wq[u].y, v[u][1], wq[u].x * v[u][0])));
                    A += col;
                    K = fmaf(kf + (float)u, col, K);
                    row[kk + u] = make_float2(A, K);
                }
            }
            tot[vw * nz + c] = make_float2(A, K);
        }
        __syncthreads();
        if (vw > 0) {
            for (int c = vl; c < nz; c += lstep) {
                float2 off = tot[c];
                for (int w2 = 1; w2 < vw; w2++) {
                    const float2 t = tot[w2 * nz + c];
                    off.x += t.x;
                    off.y += t.y;
                }
                float2 *row = tab + (c + 1) * S + 1;
                for (int kk = ka; kk < kb; kk += RB) {
                    float2 t[RB];
#pragma unroll
                    for (int u = 0; u < RB; u++) t[u] = row[kk + u];
#pragma unroll
                    for (int u = 0; u < RB; u++) row[kk + u] = make_float2(t[u].x + off.x, t[u].y + off.y);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < NPT; p++) {
            const float sa = fmaf((float)k0, dl[p], s0[p]);
            const float se = fmaf((float)(KC - 1), dl[p], sa);
            // the mirror ray's index is nz + 1 - s: both read zeros only when ray j does
            if (fmaxf(sa, se) < 0.0f || fminf(sa, se) >= (float)(tw - 1)) continue;
            const int sg = dl[p] >= 0.0f ? 1 : -1;
            float ef = floorf(sa);
            int e = (int)ef, kp = 0;
            float r = 0.0f, rm = 0.0f;
            for (;;) {
                // the runs in cell e (ray j) and cell nz - e (mirror): local samples [kp, kn)
                const int kn = max((int)fminf(ceilf((ef + bo[p] - sa) * idl[p]), (float)KC), kp);
                const int ec = min(max(e, 0), tw - 2), em = min(max(nz - e, 0), tw - 2);
                const float2 *t = tab + ec * S, *tm = tab + em * S;
                const float2 a1 = t[kn], b1 = t[kn + S], a0 = t[kp], b0 = t[kp + S];
                const float2 c1 = tm[kn], d1 = tm[kn + S], c0 = tm[kp], d0 = tm[kp + S];
                const float fe = sa - ef;
                const float dA0 = a1.x - a0.x, dA1 = b1.x - b0.x, dK0 = a1.y - a0.y, dK1 = b1.y - b0.y;
                const float run = fmaf(dl[p], dK1 - dK0, fmaf(fe, dA1 - dA0, dA0));
                // mirror: fraction 1 - fe, step -delta
                const float mA0 = c1.x - c0.x, mA1 = d1.x - d0.x, mK0 = c1.y - c0.y, mK1 = d1.y - d0.y;
                const float runm = fmaf(-dl[p], mK1 - mK0, fmaf(1.0f - fe, mA1 - mA0, mA0));
                r += (e == ec) ? run : 0.0f;
                rm += (nz - e == em) ? runm : 0.0f;
                if (kn >= KC) break;
                kp = kn;
                e += sg;
                ef += (float)sg;
            }
            acc[p] += r;
            accm[p] += rm;
        }
    }

    double part = 0.0;
#pragma unroll
    for (int p = 0; p < NPT; p++) {
        const int j = tid + p * nthr;
        if (j < npairs) {
            const int jm = nv - 1 - j;
            const float v = ((float)j - 0.5f * (float)(nv - 1)) * pv;
            const float wr = cp.wsc * sqrtf(fmaf(v, v, cp.r2));  // the mirror has the same weight
            const long o1 = ((long)view * nv + j) * nu + i, o2 = ((long)view * nv + jm) * nu + i;
            float r1 = wr * acc[p], r2 = wr * accm[p];
            if (ysub) {
                r1 -= ysub[o1];
                r2 -= ysub[o2];
                part += (double)r1 * (double)r1;
                if (jm != j) part += (double)r2 * (double)r2;
                if (wres) {
                    r1 *= wr;
                    r2 *= wr;
                }
            }
            out[o1] = r1;
            if (jm != j) out[o2] = r2;
        }
    }
    if (partials) {
        part = wave_sum(part);
        if (lane == 0) wsum[wave] = part;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w2 = 0; w2 < nw; w2++) s += wsum[w2];
            partials[(long)view * nu + i] = s;
        }
    }
}

template <int KC, int NPT>
__global__ void __launch_bounds__(256)
    k_forward_runs(const float *__restrict__ vol_t, const ColParams *__restrict__ cols, int nx, int ny, int nz, int nu,
                   int nv, float pv, const float *__restrict__ ysub, int wres, float *__restrict__ out,
                   double *__restrict__ partials) {
    // adjacent columns of one view sweep nearly the same voxels: keep them on one XCD
    const int w = cbct_xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    forward_runs_body<KC, NPT>(vol_t, cols, nx, ny, nz, nu, nv, pv, ysub, wres, out, partials, w % nu, w / nu);
}

// batched residual P (serving engine): request q owns work-groups [wg0[q], wg0[q+1]), one per
// (view, column) of its own geometry, all with the same chunk, rows per thread and block size
struct BFwItem {
    const float *vol_t;
    const ColParams *cols;
    const float *ysub;
    float *out;
    double *partials;
    int nx, ny, nz, nu, nv, nviews;
    float pv;
};
struct BFw {
    int n;
    int wg0[CBCT_MAXB + 1];
    BFwItem it[CBCT_MAXB];
};

template <int KC, int NPT>
__global__ void __launch_bounds__(256) k_forward_runs_b(BFw B) {
    int r = 0;
    while (r + 1 < B.n && (int)blockIdx.x >= B.wg0[r + 1]) r++;
    const BFwItem &it = B.it[r];
    const int w = cbct_batch_local(B.wg0[r], B.wg0[r + 1] - B.wg0[r]);
    if (w >= it.nu * it.nviews) return;  // padding
    forward_runs_body<KC, NPT>(it.vol_t, it.cols, it.nx, it.ny, it.nz, it.nu, it.nv, it.pv, it.ysub, 1, it.out,
                               it.partials, w % it.nu, w / it.nu);
}

template <int KC, int NPT>
cbct_status launch_fwd_runs_b(const BFw &B, size_t lds, int block, hipStream_t s) {
    hipLaunchKernelGGL((k_forward_runs_b<KC, NPT>), dim3(B.wg0[B.n]), dim3(block), lds, s, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_forward_runs_b launch");
    return CBCT_OK;
}

template <int KC, int NPT>
cbct_status launch_fwd_runs(const Level &L, const float *vol_t, const float *ysub, int wres, float *out,
                            double *partials, hipStream_t s, int block) {
    const size_t lds = runs_lds_bytes<KC>(L.nz, block / 64);
    dim3 grid(L.nu, L.nviews);
    hipLaunchKernelGGL((k_forward_runs<KC, NPT>), grid, dim3(block), lds, s, vol_t, L.d_cols, L.nx, L.ny, L.nz, L.nu,
                       L.nv, (float)L.pv, ysub, wres, out, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_forward_runs launch");
    return CBCT_OK;
}

template <int KC>
cbct_status dispatch_fwd_runs(const Level &L, const float *vol_t, const float *ysub, int wres, float *out,
                              double *partials, hipStream_t s, int npt, int block) {
    if (npt == 1) return launch_fwd_runs<KC, 1>(L, vol_t, ysub, wres, out, partials, s, block);
    if (npt == 2) return launch_fwd_runs<KC, 2>(L, vol_t, ysub, wres, out, partials, s, block);
    if (npt == 4) return launch_fwd_runs<KC, 4>(L, vol_t, ysub, wres, out, partials, s, block);
    if (npt == 8) return launch_fwd_runs<KC, 8>(L, vol_t, ysub, wres, out, partials, s, block);
    return cbct_set_error(CBCT_ERR_INVALID_ARG, "forward: %d detector rows is more than supported", L.nv);
}

template <int KC, int NPT, bool VEC>
cbct_status launch_fwd(const Level &L, const float *vol_t, const float *ysub, int wres, float *out, double *partials,
                       hipStream_t s, int block) {
    const size_t table = (((size_t)L.fwd_tw * (2 * KC + 1) + 3) & ~(size_t)3) * sizeof(float);
    const size_t lds = table + (size_t)KC * (sizeof(float4) + sizeof(int4));
    dim3 grid(L.nu, L.nviews);
    hipLaunchKernelGGL((k_forward<KC, NPT, VEC>), grid, dim3(block), lds, s, vol_t, L.d_cols, L.nx, L.ny, L.nz,
                       L.nu, L.nv, (float)L.pv, L.fwd_pad, L.fwd_tw, ysub, wres, out, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_forward launch");
    return CBCT_OK;
}

}  // namespace

cbct_status cbct_launch_to_columns(const Level &L, const float *vol, float *vol_t, hipStream_t s) {
    dim3 grid((L.nx + 31) / 32, (L.nz + 31) / 32, L.ny);
    hipLaunchKernelGGL(k_to_columns, grid, dim3(32, 8), 0, s, vol, vol_t, L.nx, L.ny, L.nz);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_to_columns launch");
    return CBCT_OK;
}

int cbct_forward_runs_block(int nv, int *npt) {
    const int npairs = (nv + 1) / 2;
    int n = 1;
    while ((npairs + n - 1) / n > 256) n *= 2;
    if (npt) *npt = n;
    return (((npairs + n - 1) / n + 63) / 64) * 64;
}

// The chunk (samples per table).  One-wave work-groups (up to 128 detector rows) take 16 samples
// (8 where those tables do not fit 48 KB): with no build to split, the most work-groups per CU win.
// With two or more waves, which split each chunk's build into slices of whole groups of 8 samples,
// the largest multiple of 8 from 64 down to 16 whose tables leave LDS for six work-groups per CU
// (160 KB / 6); where none does (depths above 157), the largest of 64, 32 or 16 within 32 KB, else
// the largest of 64, 32, 16 or 8 within 48 KB.  The projector lives on occupancy and on the
// build's balance over the waves: at 512x512x64 / 40 views (three waves) 40 samples, slices of 16,
// 16 and 8 at six work-groups per CU, took 0.74-0.76 ms per P against 0.77-0.78 with 48 (balanced,
// five per CU), 0.79-0.81 with 32 (slices 16, 16 and none) and 0.84 with 24; at 256x256x96 / 82
// views (two waves) 24 samples took 1.13 against 1.32 ms with 32; one-wave 64^3 / 77 views took
// 0.043 ms with 16 against 0.046 with 24 and 0.054 with 32, and 32^3 / 16 views 0.010 against
// 0.012 ms with 64; at 128^3 / 60 views 16-sample chunks, eight work-groups per CU, took 0.25 ms
// against 0.30 with 32 at four per CU and 0.56 with 64 at two.
int cbct_forward_run_chunk(int nz, int nwaves) {
    constexpr size_t six = 160 * 1024 / 6, small = 32 * 1024, budget = 48 * 1024;
    if (nwaves == 1) {
        if (runs_lds_bytes_kc(16, nz, 4) <= budget) return 16;
        return runs_lds_bytes_kc(8, nz, 4) <= budget ? 8 : 0;
    }
    for (int kc = 64; kc >= 16; kc -= 8)
        if (runs_lds_bytes_kc(kc, nz, 4) <= six) return kc;
    for (int kc = 64; kc >= 16; kc /= 2)
        if (runs_lds_bytes_kc(kc, nz, 4) <= small) return kc;
    for (int kc = 64; kc >= 8; kc /= 2)
        if (runs_lds_bytes_kc(kc, nz, 4) <= budget) return kc;
    return 0;
}

cbct_status cbct_launch_forward(const Level &L, const float *vol_t, const float *ysub, float *out, double *partials,
                                hipStream_t s, bool weight_residual) {
    const int wres = weight_residual ? 1 : 0;
    if (L.fwd_kr > 0) {
        // rays per thread and a work-group size that splits the rows evenly
        int npt = 1;
        const int block = cbct_forward_runs_block(L.nv, &npt);
        switch (L.fwd_kr) {
#define CBCT_FWR(KC_) \
    case KC_: return dispatch_fwd_runs<KC_>(L, vol_t, ysub, wres, out, partials, s, npt, block);
            CBCT_FWR(64) CBCT_FWR(56) CBCT_FWR(48) CBCT_FWR(40) CBCT_FWR(32) CBCT_FWR(24) CBCT_FWR(16) CBCT_FWR(8)
#undef CBCT_FWR
            default: return cbct_set_error(CBCT_ERR_INTERNAL, "forward: unsupported chunk %d", L.fwd_kr);
        }
    }
    const int npairs = (L.nv + 1) / 2;
    int block = ((npairs + 63) / 64) * 64;
    int npt = 1;
    while (block > 256) {
        npt *= 2;
        block = ((((npairs + npt - 1) / npt) + 63) / 64) * 64;
    }
    if (L.fwd_kc > block)
        return cbct_set_error(CBCT_ERR_INTERNAL, "forward: chunk %d larger than the work-group %d", L.fwd_kc, block);
    const bool vec = (L.nz % 4) == 0;
#define CBCT_FWD(KC_, NPT_)                                                                     \
    return vec ? launch_fwd<KC_, NPT_, true>(L, vol_t, ysub, wres, out, partials, s, block)      \
               : launch_fwd<KC_, NPT_, false>(L, vol_t, ysub, wres, out, partials, s, block)
    if (L.fwd_kc == 32) {
        if (npt == 1) CBCT_FWD(32, 1);
        if (npt == 2) CBCT_FWD(32, 2);
        if (npt == 4) CBCT_FWD(32, 4);
    } else if (L.fwd_kc == 16) {
        if (npt == 1) CBCT_FWD(16, 1);
        if (npt == 2) CBCT_FWD(16, 2);
        if (npt == 4) CBCT_FWD(16, 4);
    } else {
        return cbct_set_error(CBCT_ERR_INTERNAL, "forward: unsupported chunk %d", L.fwd_kc);
    }
#undef CBCT_FWD
    return cbct_set_error(CBCT_ERR_INVALID_ARG, "forward: %d detector rows is more than supported", L.nv);
}

// the run-summing projector's configuration of a level: chunk, row pairs per thread, block size
static bool fwd_runs_config(const Level &L, int &kc, int &npt, int &block) {
    if (L.fwd_kr <= 0) return false;
    block = cbct_forward_runs_block(L.nv, &npt);
    kc = L.fwd_kr;
    return npt <= 8;
}

cbct_status cbct_launch_forward_batch(const FwdReq *r, int n, hipStream_t s) {
    std::vector<bool> done(n, false);
    for (int q = 0; q < n; q++) {
        if (done[q]) continue;
        int kc, npt, block;
        if (!fwd_runs_config(*r[q].L, kc, npt, block)) {
            // per-sample projector: a launch of its own
            done[q] = true;
            cbct_status st = cbct_launch_forward(*r[q].L, r[q].vol_t, r[q].ysub, r[q].out, r[q].partials, s, true);
            if (st) return st;
            continue;
        }
        // every remaining request with the same configuration, up to CBCT_MAXB per launch
        BFw B{};
        size_t lds = 0;
        int w = 0;
        for (int q2 = q; q2 < n && B.n < CBCT_MAXB; q2++) {
            int kc2, npt2, block2;
            if (done[q2] || !fwd_runs_config(*r[q2].L, kc2, npt2, block2) || kc2 != kc || npt2 != npt ||
                block2 != block)
                continue;
            done[q2] = true;
            const Level &L = *r[q2].L;
            B.it[B.n] = BFwItem{r[q2].vol_t, L.d_cols, r[q2].ysub, r[q2].out, r[q2].partials, L.nx, L.ny, L.nz,
                                L.nu, L.nv, L.nviews, (float)L.pv};
            B.wg0[B.n] = w;
            w += cbct_batch_pad(L.nu * L.nviews);
            B.n++;
            lds = std::max(lds, runs_lds_bytes_kc(kc, L.nz, block / 64));
        }
        B.wg0[B.n] = w;
        cbct_status st = CBCT_OK;
#define CBCT_FWB(KC_)                                                           \
    if (npt == 1) st = launch_fwd_runs_b<KC_, 1>(B, lds, block, s);             \
    else if (npt == 2) st = launch_fwd_runs_b<KC_, 2>(B, lds, block, s);        \
    else if (npt == 4) st = launch_fwd_runs_b<KC_, 4>(B, lds, block, s);        \
    else st = launch_fwd_runs_b<KC_, 8>(B, lds, block, s);
        switch (kc) {
            case 64: CBCT_FWB(64) break;
            case 56: CBCT_FWB(56) break;
            case 48: CBCT_FWB(48) break;
            case 40: CBCT_FWB(40) break;
            case 32: CBCT_FWB(32) break;
            case 24: CBCT_FWB(24) break;
            case 16: CBCT_FWB(16) break;
            case 8: CBCT_FWB(8) break;
            default: st = cbct_set_error(CBCT_ERR_INTERNAL, "forward: unsupported chunk %d", kc);
        }
#undef CBCT_FWB
        if (st) return st;
    }
    return CBCT_OK;
}
