// Multigrid transfers (Section II.C.3 of the paper: solve on the coarser grid, extend the
// solution smoothly to the finer grid as its initial guess) and small vector kernels.
//
// Prolongation is cell-centred trilinear: fine cell F along an axis takes 3/4 of its parent
// F/2 and 1/4 of the parent's neighbour on F's side (index clamped at the ends).  Restriction is
// (1/8) Prol^T.  The detector pyramid is a 2^l x 2^l block mean.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>

#include "cbct_internal.h"

namespace {

// the two coarse samples of fine index F (n coarse samples) and their weights
__device__ __forceinline__ void prol_taps(int F, int n, int &i0, int &i1, float &w0, float &w1) {
    const int p = F >> 1;
    int q = (F & 1) ? p + 1 : p - 1;
    q = min(max(q, 0), n - 1);
    i0 = p;
    i1 = q;
    if (q == p) {
        w0 = 1.0f;
        w1 = 0.0f;
    } else {
        w0 = 0.75f;
        w1 = 0.25f;
    }
}

// weight of coarse index c in fine index F (0 if c is not one of F's taps)
__device__ __forceinline__ float prol_w(int F, int c, int n) {
    int i0, i1;
    float w0, w1;
    prol_taps(F, n, i0, i1, w0, w1);
    return (c == i0 ? w0 : 0.0f) + (c == i1 ? w1 : 0.0f);
}

__global__ void __launch_bounds__(256) k_prolong(const float *__restrict__ c, float *__restrict__ f, int nx, int ny,
                                                 int nz) {
    const int NX = 2 * nx, NY = 2 * ny, NZ = 2 * nz;
    const long n = (long)NX * NY * NZ;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x) {
        const int A = (int)(p % NX), B = (int)((p / NX) % NY), C = (int)(p / ((long)NX * NY));
        int x0, x1, y0, y1, z0, z1;
        float wx0, wx1, wy0, wy1, wz0, wz1;
        prol_taps(A, nx, x0, x1, wx0, wx1);
        prol_taps(B, ny, y0, y1, wy0, wy1);
        prol_taps(C, nz, z0, z1, wz0, wz1);
        auto at = [&](int z, int y, int x) { return c[((long)z * ny + y) * nx + x]; };
        const float a0 = wx0 * at(z0, y0, x0) + wx1 * at(z0, y0, x1);
        const float a1 = wx0 * at(z0, y1, x0) + wx1 * at(z0, y1, x1);
        const float b0 = wx0 * at(z1, y0, x0) + wx1 * at(z1, y0, x1);
        const float b1 = wx0 * at(z1, y1, x0) + wx1 * at(z1, y1, x1);
        f[p] = wz0 * (wy0 * a0 + wy1 * a1) + wz1 * (wy0 * b0 + wy1 * b1);
    }
}

__global__ void __launch_bounds__(256) k_restrict(const float *__restrict__ f, float *__restrict__ c, int nx, int ny,
                                                  int nz) {
    const int NX = 2 * nx, NY = 2 * ny, NZ = 2 * nz;
    const long n = (long)nx * ny * nz;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x) {
        const int a = (int)(p % nx), b = (int)((p / nx) % ny), cc = (int)(p / ((long)nx * ny));
        float s = 0.0f;
        for (int Z = max(2 * cc - 1, 0); Z <= min(2 * cc + 2, NZ - 1); Z++) {
            const float wz = prol_w(Z, cc, nz);
            if (wz == 0.0f) continue;
            for (int Y = max(2 * b - 1, 0); Y <= min(2 * b + 2, NY - 1); Y++) {
                const float wy = prol_w(Y, b, ny);
                if (wy == 0.0f) continue;
                float row = 0.0f;
                for (int X = max(2 * a - 1, 0); X <= min(2 * a + 2, NX - 1); X++)
                    row += prol_w(X, a, nx) * f[((long)Z * NY + Y) * NX + X];
                s += wz * wy * row;
            }
        }
        c[p] = 0.125f * s;
    }
}

__global__ void __launch_bounds__(256) k_bin(const float *__restrict__ y0, float *__restrict__ yl, int nviews, int nv,
                                             int nu, int fct) {
    const int mv = nv / fct, mu = nu / fct;
    const long n = (long)nviews * mv * mu;
    const float inv = 1.0f / (float)(fct * fct);
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x) {
        const int i = (int)(p % mu), j = (int)((p / mu) % mv), v = (int)(p / ((long)mu * mv));
        float s = 0.0f;
        for (int jj = 0; jj < fct; jj++)
            for (int ii = 0; ii < fct; ii++) s += y0[((long)v * nv + j * fct + jj) * nu + i * fct + ii];
        yl[p] = s * inv;
    }
}

// Step 3 (f = max(u, 0)) fused with the copy of f into the projector's column-major layout
__device__ __forceinline__ void clamp_columns_body(const float *__restrict__ u, const float *__restrict__ d,
                                                   const RofControl *__restrict__ ctl, float *__restrict__ f,
                                                   float *__restrict__ f_t, int nx, int ny, int nz, int bx, int by,
                                                   int bz) {
    __shared__ float tile[32][33];
    // a pending accepted ROF step u - s d is applied here (the same product as the update kernel's)
    const bool step = d && ctl->accepted == 1;
    const float st = step ? (float)ctl->s : 0.0f;
    const int b = bz;
    const int a0 = bx * 32, c0 = by * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;
    for (int r = ty; r < 32; r += 8) {
        const int c = c0 + r, a = a0 + tx;
        if (c < nz && a < nx) {
            const long p = ((long)c * ny + b) * nx + a;
            const float v = fmaxf(step ? fmaf(-st, d[p], u[p]) : u[p], 0.0f);
            f[p] = v;
            tile[r][tx] = v;
        }
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int a = a0 + r, c = c0 + tx;
        if (a < nx && c < nz) f_t[((long)b * nx + a) * nz + c] = tile[tx][r];
    }
}

__global__ void __launch_bounds__(256) k_clamp_columns(const float *__restrict__ u, const float *__restrict__ d,
                                                       const RofControl *__restrict__ ctl, float *__restrict__ f,
                                                       float *__restrict__ f_t, int nx, int ny, int nz) {
    clamp_columns_body(u, d, ctl, f, f_t, nx, ny, nz, blockIdx.x, blockIdx.y, blockIdx.z);
}

// batched Step 3 (serving engine): request q owns work-groups [wg0[q], wg0[q+1]) of a flat grid,
// each running the solo kernel's body at its place in the request's (nx/32, nz/32, ny) grid
struct BClItem {
    const float *u, *d;
    const RofControl *ctl;
    float *f, *f_t;
    int nx, ny, nz, gx, gy;
};
struct BCl {
    int n;
    int wg0[CBCT_MAXB + 1];
    BClItem it[CBCT_MAXB];
};

__global__ void __launch_bounds__(256) k_clamp_columns_b(BCl B) {
    int r = 0;
    while (r + 1 < B.n && (int)blockIdx.x >= B.wg0[r + 1]) r++;
    const BClItem &it = B.it[r];
    const int local = blockIdx.x - B.wg0[r];
    const int bx = local % it.gx, rest = local / it.gx;
    clamp_columns_body(it.u, it.d, it.ctl, it.f, it.f_t, it.nx, it.ny, it.nz, bx, rest % it.gy, rest / it.gy);
}

__global__ void k_fill(float *__restrict__ x, long n, float v) {
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x) x[p] = v;
}

__global__ void __launch_bounds__(256) k_max_part(const float *__restrict__ x, long n, double *__restrict__ part) {
    __shared__ float sh[256];
    float m = -FLT_MAX;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x)
        m = fmaxf(m, x[p]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = (double)sh[0];
}

// max is exact and order-free, so the split over threads keeps the result deterministic
__global__ void __launch_bounds__(256) k_max_final(const double *__restrict__ part, int nb, double *__restrict__ out) {
    __shared__ double sh[256];
    double m = -1e300;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) m = fmax(m, part[b]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

int grid_for(long n) { return (int)std::min<long>(std::max<long>((n + 255) / 256, 1), 8192); }

}  // namespace

#define LAUNCH_CHECK(what)                                     \
    do {                                                       \
        hipError_t e_ = hipGetLastError();                     \
        if (e_ != hipSuccess) return cbct_hip_error(e_, what); \
    } while (0)

cbct_status cbct_launch_prolong(const Level &coarse, const float *c, float *f, hipStream_t s) {
    hipLaunchKernelGGL(k_prolong, dim3(grid_for(coarse.nvox() * 8)), dim3(256), 0, s, c, f, coarse.nx, coarse.ny,
                       coarse.nz);
    LAUNCH_CHECK("k_prolong");
    return CBCT_OK;
}

cbct_status cbct_launch_restrict(const Level &coarse, const float *f, float *c, hipStream_t s) {
    hipLaunchKernelGGL(k_restrict, dim3(grid_for(coarse.nvox())), dim3(256), 0, s, f, c, coarse.nx, coarse.ny,
                       coarse.nz);
    LAUNCH_CHECK("k_restrict");
    return CBCT_OK;
}

cbct_status cbct_launch_bin(const Level &fine0, int factor, const float *y0, float *yl, hipStream_t s) {
    const long n = (long)fine0.nviews * (fine0.nv / factor) * (fine0.nu / factor);
    hipLaunchKernelGGL(k_bin, dim3(grid_for(n)), dim3(256), 0, s, y0, yl, fine0.nviews, fine0.nv, fine0.nu, factor);
    LAUNCH_CHECK("k_bin");
    return CBCT_OK;
}

cbct_status cbct_launch_clamp_columns(const Level &L, const float *u, float *f, float *f_t, hipStream_t s,
                                      const float *d, const RofControl *ctl) {
    dim3 grid((L.nx + 31) / 32, (L.nz + 31) / 32, L.ny);
    hipLaunchKernelGGL(k_clamp_columns, grid, dim3(32, 8), 0, s, u, d, ctl, f, f_t, L.nx, L.ny, L.nz);
    LAUNCH_CHECK("k_clamp_columns");
    return CBCT_OK;
}

cbct_status cbct_launch_fill(float *x, long n, float v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, x, n, v);
    LAUNCH_CHECK("k_fill");
    return CBCT_OK;
}

cbct_status cbct_launch_max(const float *x, long n, double *partials, double *out, hipStream_t s) {
    const int nb = (int)std::min<long>(std::max<long>((n + 255) / 256, 1), CBCT_RED_BLOCKS);
    hipLaunchKernelGGL(k_max_part, dim3(nb), dim3(256), 0, s, x, n, partials);
    LAUNCH_CHECK("k_max_part");
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, partials, nb, out);
    LAUNCH_CHECK("k_max_final");
    return CBCT_OK;
}

cbct_status cbct_launch_clamp_batch(const ClampReq *r, int n, hipStream_t s) {
    for (int q0 = 0; q0 < n; q0 += CBCT_MAXB) {
        const int m = std::min(CBCT_MAXB, n - q0);
        BCl B{};
        B.n = m;
        int w = 0;
        for (int q = 0; q < m; q++) {
            const ClampReq &c = r[q0 + q];
            const Level &L = *c.L;
            const int gx = (L.nx + 31) / 32, gy = (L.nz + 31) / 32;
            B.it[q] = BClItem{c.u, c.d, c.ctl, c.f, c.f_t, L.nx, L.ny, L.nz, gx, gy};
            B.wg0[q] = w;
            w += gx * gy * L.ny;
        }
        B.wg0[m] = w;
        hipLaunchKernelGGL(k_clamp_columns_b, dim3(w), dim3(32, 8), 0, s, B);
        LAUNCH_CHECK("k_clamp_columns_b");
    }
    return CBCT_OK;
}
