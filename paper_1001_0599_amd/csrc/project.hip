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

cbct_status cbct_launch_forward(const Level &L, const float *vol_t, const float *ysub, float *out, double *partials,
                                hipStream_t s, bool weight_residual) {
    const int wres = weight_residual ? 1 : 0;
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
