// TV / ROF kernels (Step 2 of Algorithm A1, Eq. 5 of the paper) and the deterministic
// reductions behind the Armijo decisions.
//
// Volumes are [nz][ny][nx] (x fastest).  Smoothed TV with the paper's boundary conditions:
// forward differences, ghost 0 beyond the last x and y sample (zero BC, lateral and AP), ghost
// = last plane beyond the last z plane (reflective, superior-inferior).  Per voxel
//   phi(p) = sqrt(|D u(p)|^2 + eps^2),  q(p) = D u(p) / phi(p),
//   R(u) = mean phi,  N dR/du_p = sum_d (q_d(p - e_d) [p - e_d in grid] - q_d(p)) / h_d.
// The ROF energy E_R(u) = lambda R(u) + mean((u-g)^2) / (2t) and its normalised gradient
// d = lambda N dR/du + (u-g)/t are produced by one stencil pass (13 reads per voxel, served by
// L1/L2; HBM sees u, g in and d out).  Trial energies E_R(u - s_m d) for M step sizes
// s_m = t alpha^m come from one more pass, so one pass covers several backtracking steps.
//
// Every reduction is two-level and fixed-order: each work-group of a fixed-size grid writes
// FP64 partial sums, and a single-work-group kernel sums them in order, so results are
// bitwise reproducible and independent of timing.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cbct_internal.h"

namespace {

struct TVShape {
    int nx, ny, nz;
    float ihx, ihy, ihz, eps2;
};

__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); k++) s += sh[k];
    return s;  // valid in thread 0
}

// forward differences of v at p = (a, b, c)
__device__ __forceinline__ void diffs(const float *__restrict__ v, long p, int a, int b, int c, const TVShape &k,
                                      float &dx, float &dy, float &dz) {
    const long nxy = (long)k.nx * k.ny;
    const float v0 = v[p];
    const float vx = (a + 1 < k.nx) ? v[p + 1] : 0.0f;
    const float vy = (b + 1 < k.ny) ? v[p + k.nx] : 0.0f;
    const float vz = (c + 1 < k.nz) ? v[p + nxy] : v0;
    dx = (vx - v0) * k.ihx;
    dy = (vy - v0) * k.ihy;
    dz = (vz - v0) * k.ihz;
}

// differences of w = u - s d at p
__device__ __forceinline__ void diffs_step(const float *__restrict__ u, const float *__restrict__ d, float s, long p,
                                           int a, int b, int c, const TVShape &k, float &w0, float &dx, float &dy,
                                           float &dz) {
    const long nxy = (long)k.nx * k.ny;
    w0 = fmaf(-s, d[p], u[p]);
    const float wx = (a + 1 < k.nx) ? fmaf(-s, d[p + 1], u[p + 1]) : 0.0f;
    const float wy = (b + 1 < k.ny) ? fmaf(-s, d[p + k.nx], u[p + k.nx]) : 0.0f;
    const float wz = (c + 1 < k.nz) ? fmaf(-s, d[p + nxy], u[p + nxy]) : w0;
    dx = (wx - w0) * k.ihx;
    dy = (wy - w0) * k.ihy;
    dz = (wz - w0) * k.ihz;
}

__device__ __forceinline__ float phi_of(float dx, float dy, float dz, float eps2) {
    // hardware square root (1 ulp): the argument is at least eps^2, a normal number
    return __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2))));
}

// Work distribution of the TV kernels: lanes run along x (64 per row segment), work-groups take
// (row segment, 4 rows) tiles and stride over the (y, z) rows, so there is one division per row
// and the grid (hence the partial-sum layout) is fixed by the shape.
struct RowIter {
    int nrow, row0, rstep, a0, astep;
};

__device__ __forceinline__ RowIter row_iter(const TVShape &k) {
    RowIter it;
    it.nrow = k.ny * k.nz;
    it.row0 = blockIdx.y * 4 + (threadIdx.x >> 6);
    it.rstep = gridDim.y * 4;
    it.a0 = blockIdx.x * 64 + (threadIdx.x & 63);
    it.astep = gridDim.x * 64;
    return it;
}

// d = lambda * N dR/du + (u - g)/t (g may be NULL: then d = N dR/du and lambda is ignored).
// partials[block] = {sum phi, sum (u-g)^2, sum d^2}.
__global__ void __launch_bounds__(256) k_tv_grad(const float *__restrict__ u, const float *__restrict__ g,
                                                 float *__restrict__ d, TVShape k, float lambda, float inv_t,
                                                 double *__restrict__ partials) {
    __shared__ double sh[4];
    const long nxy = (long)k.nx * k.ny;
    double s_phi = 0.0, s_fid = 0.0, s_d2 = 0.0;
    const RowIter ri = row_iter(k);
    for (int row = ri.row0; row < ri.nrow; row += ri.rstep) {
        const int c = row / k.ny, b = row - c * k.ny;
        const long rbase = (long)c * nxy + (long)b * k.nx;
        for (int a = ri.a0; a < k.nx; a += ri.astep) {
            const long p = rbase + a;
            float dx, dy, dz;
            diffs(u, p, a, b, c, k, dx, dy, dz);
            const float ph = phi_of(dx, dy, dz, k.eps2);
            const float ip = __builtin_amdgcn_rcpf(ph);  // 1 ulp reciprocals instead of divisions
            // the z difference of the last plane is identically 0 (reflective ghost): q_z = 0 there
            float div = -(dx * ip * k.ihx + dy * ip * k.ihy + dz * ip * k.ihz);
            if (a >= 1) {
                float ex, ey, ez;
                diffs(u, p - 1, a - 1, b, c, k, ex, ey, ez);
                div += ex * __builtin_amdgcn_rcpf(phi_of(ex, ey, ez, k.eps2)) * k.ihx;
            }
            if (b >= 1) {
                float ex, ey, ez;
                diffs(u, p - k.nx, a, b - 1, c, k, ex, ey, ez);
                div += ey * __builtin_amdgcn_rcpf(phi_of(ex, ey, ez, k.eps2)) * k.ihy;
            }
            if (c >= 1) {
                float ex, ey, ez;
                diffs(u, p - nxy, a, b, c - 1, k, ex, ey, ez);
                div += ez * __builtin_amdgcn_rcpf(phi_of(ex, ey, ez, k.eps2)) * k.ihz;
            }
            float dv;
            if (g) {
                const float r = u[p] - g[p];
                dv = fmaf(lambda, div, r * inv_t);
                s_fid += (double)r * (double)r;
            } else {
                dv = div;
            }
            d[p] = dv;
            s_phi += (double)ph;
            s_d2 += (double)dv * (double)dv;
        }
    }
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
    double v;
    v = block_sum(s_phi, sh);
    if (threadIdx.x == 0) partials[blk * 3 + 0] = v;
    v = block_sum(s_fid, sh);
    if (threadIdx.x == 0) partials[blk * 3 + 1] = v;
    v = block_sum(s_d2, sh);
    if (threadIdx.x == 0) partials[blk * 3 + 2] = v;
}

// sum phi only (energy of a volume)
__global__ void __launch_bounds__(256) k_tv_energy(const float *__restrict__ u, TVShape k,
                                                   double *__restrict__ partials) {
    __shared__ double sh[4];
    const long nxy = (long)k.nx * k.ny;
    double s_phi = 0.0;
    const RowIter ri = row_iter(k);
    for (int row = ri.row0; row < ri.nrow; row += ri.rstep) {
        const int c = row / k.ny, b = row - c * k.ny;
        const long rbase = (long)c * nxy + (long)b * k.nx;
        for (int a = ri.a0; a < k.nx; a += ri.astep) {
            float dx, dy, dz;
            diffs(u, rbase + a, a, b, c, k, dx, dy, dz);
            s_phi += (double)phi_of(dx, dy, dz, k.eps2);
        }
    }
    const double v = block_sum(s_phi, sh);
    if (threadIdx.x == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = v;
}

// Trial energies at s_m = s0 * alpha^m, m < M.  partials[block][2m + {0,1}] = {sum phi, sum fid}.
template <int M>
__global__ void __launch_bounds__(256) k_tv_trial(const float *__restrict__ u, const float *__restrict__ d,
                                                  const float *__restrict__ g, TVShape k, double t, double alpha,
                                                  int m0, double *__restrict__ partials) {
    __shared__ double sh[4];
    const long nxy = (long)k.nx * k.ny;
    // s_m = t alpha^(m0 + m), formed exactly as the decision kernel forms it
    float s[M];
    double sd = t;
    for (int m = 0; m < m0; m++) sd *= alpha;
#pragma unroll
    for (int m = 0; m < M; m++) {
        s[m] = (float)sd;
        sd *= alpha;
    }
    double s_phi[M], s_fid[M];
#pragma unroll
    for (int m = 0; m < M; m++) s_phi[m] = s_fid[m] = 0.0;
    const RowIter ri = row_iter(k);
    for (int row = ri.row0; row < ri.nrow; row += ri.rstep) {
        const int c = row / k.ny, b = row - c * k.ny;
        const long rbase = (long)c * nxy + (long)b * k.nx;
        for (int a = ri.a0; a < k.nx; a += ri.astep) {
            const long p = rbase + a;
            const float gp = g[p];
#pragma unroll
            for (int m = 0; m < M; m++) {
                float w0, dx, dy, dz;
                diffs_step(u, d, s[m], p, a, b, c, k, w0, dx, dy, dz);
                const float r = w0 - gp;
                s_phi[m] += (double)phi_of(dx, dy, dz, k.eps2);
                s_fid[m] += (double)r * (double)r;
            }
        }
    }
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
    for (int m = 0; m < M; m++) {
        double v = block_sum(s_phi[m], sh);
        if (threadIdx.x == 0) partials[blk * 2 * M + 2 * m] = v;
        v = block_sum(s_fid[m], sh);
        if (threadIdx.x == 0) partials[blk * 2 * M + 2 * m + 1] = v;
    }
}

// sum of `nb` rows of `width` partials: out[j] = sum_b part[b * width + j], in a fixed order
// (each thread sums a contiguous run of rows, then a fixed binary tree over the threads), so the
// result does not depend on timing
constexpr int SUM_MAXW = 3 + 2 * CBCT_TRIALS;
__global__ void __launch_bounds__(256) k_sum_rows(const double *__restrict__ part, int nb, int width,
                                                  double *__restrict__ out) {
    __shared__ double sh[SUM_MAXW][256];
    const int per = (nb + blockDim.x - 1) / blockDim.x;
    const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    double s[SUM_MAXW];
#pragma unroll
    for (int j = 0; j < SUM_MAXW; j++) s[j] = 0.0;
    for (int b = b0; b < b1; b++) {
#pragma unroll
        for (int j = 0; j < SUM_MAXW; j++)
            if (j < width) s[j] += part[(long)b * width + j];
    }
#pragma unroll
    for (int j = 0; j < SUM_MAXW; j++)
        if (j < width) sh[j][threadIdx.x] = s[j];
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int j = 0; j < width; j++) sh[j][threadIdx.x] += sh[j][threadIdx.x + o];
        __syncthreads();
    }
    if ((int)threadIdx.x < width) out[threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_axpy_step(float *__restrict__ u, const float *__restrict__ d, const RofControl *__restrict__ ctl,
                            long n) {
    if (ctl->accepted != 1) return;
    const float s = (float)ctl->s;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x)
        u[p] = fmaf(-s, d[p], u[p]);
}

// Armijo decision for one ROF iteration from the reduced sums.
// sums: [0..2] = {sum phi(u), sum (u-g)^2, sum d^2}, [3 + 2m + {0,1}] = trial sums for m - m0.
// The record goes to ctl (read by the update kernel) and, when given, to a host-mapped mirror
// (no copy command): its fields first, then, after a system-scope fence, the call's sequence
// number in `pad`, so that a host that sees the number also sees the fields.
__global__ void k_rof_decide(const double *__restrict__ sums, int M, int m0, int forced_m, double inv_n, double lambda,
                             double t, double c_armijo, double alpha, int max_bt, RofControl *__restrict__ ctl,
                             RofControl *__restrict__ mirror, int seq) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    RofControl r{};
    r.e0 = lambda * sums[0] * inv_n + sums[1] * inv_n / (2.0 * t);
    r.G = sums[2] * inv_n;
    r.accepted = 0;
    r.next_m0 = -1;
    double s = t;
    for (int m = 0; m < m0; m++) s *= alpha;
    bool done = false;
    for (int q = 0; q < M && m0 + q <= max_bt && !done; q++) {
        const int m = m0 + q;
        const double e = lambda * sums[3 + 2 * q] * inv_n + sums[3 + 2 * q + 1] * inv_n / (2.0 * t);
        r.e_trial = e;
        r.m = m;
        r.s = s;
        const bool ok = (forced_m >= 0) ? (m == forced_m) : (e <= r.e0 - c_armijo * s * r.G);
        if (ok) {
            r.accepted = 1;
            done = true;
        }
        s *= alpha;
    }
    if (!done) {
        // none of this window satisfied the test: search further or give up
        if (m0 + M <= max_bt && (forced_m < 0 || forced_m >= m0 + M)) r.next_m0 = m0 + M;
        else r.accepted = -1;
    }
    *ctl = r;
    if (mirror) {
        r.pad = 0;
        *mirror = r;
        __threadfence_system();
        *reinterpret_cast<volatile int *>(&mirror->pad) = seq;
    }
}

}  // namespace

// ---- launchers ---------------------------------------------------------------------------
static TVShape tv_shape(const Level &L, double eps) {
    return TVShape{L.nx, L.ny, L.nz, (float)(1.0 / L.hx), (float)(1.0 / L.hy), (float)(1.0 / L.hz),
                   (float)(eps * eps)};
}

// fixed reduction grid of a volume: (x segments of 64) x (row groups of 4), about
// CBCT_RED_BLOCKS work-groups
static dim3 tv_grid(const Level &L) {
    const int gx = (L.nx + 63) / 64;
    const int rows = (L.ny * L.nz + 3) / 4;
    const int gy = std::max(1, std::min(rows, CBCT_RED_BLOCKS / gx));
    return dim3(gx, gy);
}

int cbct_reduce_blocks(const Level &L) {
    const dim3 g = tv_grid(L);
    return (int)(g.x * g.y);
}

#define LAUNCH_CHECK(what)                                  \
    do {                                                    \
        hipError_t e_ = hipGetLastError();                  \
        if (e_ != hipSuccess) return cbct_hip_error(e_, what); \
    } while (0)

cbct_status cbct_launch_tv_grad(const Level &L, double eps, const float *u, const float *g, float *d, double lambda,
                                double t, double *partials, double *sums, hipStream_t s) {
    const int nb = cbct_reduce_blocks(L);
    hipLaunchKernelGGL(k_tv_grad, tv_grid(L), dim3(256), 0, s, u, g, d, tv_shape(L, eps), (float)lambda,
                       (float)(1.0 / t), partials);
    LAUNCH_CHECK("k_tv_grad");
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, partials, nb, 3, sums);
    LAUNCH_CHECK("k_sum_rows");
    return CBCT_OK;
}

cbct_status cbct_launch_tv_energy(const Level &L, double eps, const float *u, double *partials, double *sum,
                                  hipStream_t s) {
    const int nb = cbct_reduce_blocks(L);
    hipLaunchKernelGGL(k_tv_energy, tv_grid(L), dim3(256), 0, s, u, tv_shape(L, eps), partials);
    LAUNCH_CHECK("k_tv_energy");
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, partials, nb, 1, sum);
    LAUNCH_CHECK("k_sum_rows");
    return CBCT_OK;
}

cbct_status cbct_launch_tv_trial(const Level &L, double eps, const float *u, const float *d, const float *g,
                                 double t, double alpha, int m0, int M, double *partials, double *sums, hipStream_t s) {
    const int nb = cbct_reduce_blocks(L);
    if (M == 1)
        hipLaunchKernelGGL((k_tv_trial<1>), tv_grid(L), dim3(256), 0, s, u, d, g, tv_shape(L, eps), t, alpha, m0,
                           partials);
    else
        hipLaunchKernelGGL((k_tv_trial<CBCT_TRIALS>), tv_grid(L), dim3(256), 0, s, u, d, g, tv_shape(L, eps), t,
                           alpha, m0, partials);
    LAUNCH_CHECK("k_tv_trial");
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, partials, nb, 2 * (M == 1 ? 1 : CBCT_TRIALS), sums);
    LAUNCH_CHECK("k_sum_rows");
    return CBCT_OK;
}

cbct_status cbct_launch_rof_decide(const double *sums, int m0, int M, int forced_m, long nvox, double lambda,
                                   double t, double c_armijo, double alpha, int max_bt, RofControl *ctl,
                                   RofControl *mirror, int seq, hipStream_t s) {
    hipLaunchKernelGGL(k_rof_decide, dim3(1), dim3(64), 0, s, sums, M, m0, forced_m, 1.0 / (double)nvox, lambda, t,
                       c_armijo, alpha, max_bt, ctl, mirror, seq);
    LAUNCH_CHECK("k_rof_decide");
    return CBCT_OK;
}

cbct_status cbct_launch_axpy_step(float *u, const float *d, const RofControl *ctl, long n, hipStream_t s) {
    const int nb = (int)std::min<long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_axpy_step, dim3(nb), dim3(256), 0, s, u, d, ctl, n);
    LAUNCH_CHECK("k_axpy_step");
    return CBCT_OK;
}

cbct_status cbct_launch_sum_rows(const double *part, int nb, int width, double *out, hipStream_t s) {
    if (width < 1 || width > SUM_MAXW) return cbct_set_error(CBCT_ERR_INVALID_ARG, "sum_rows: width %d", width);
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, part, nb, width, out);
    LAUNCH_CHECK("k_sum_rows");
    return CBCT_OK;
}
