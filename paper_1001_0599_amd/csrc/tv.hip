// TV / ROF kernels (Step 2 of Algorithm A1, Eq. 5 of the paper) and the deterministic
// reductions behind the Armijo decisions.
//
// Volumes are [nz][ny][nx] (x fastest).  Smoothed TV with the paper's boundary conditions:
// forward differences, ghost 0 beyond the last x and y sample (zero BC, lateral and AP), ghost
// = last plane beyond the last z plane (reflective, superior-inferior).  Per voxel
//   phi(p) = sqrt(|D u(p)|^2 + eps^2),  q(p) = D u(p) / phi(p),
//   R(u) = mean phi,  N dR/du_p = sum_d (q_d(p - e_d) [p - e_d in grid] - q_d(p)) / h_d.
// The ROF energy E_R(u) = lambda R(u) + mean((u-g)^2) / (2t) and its normalised gradient
// d = lambda N dR/du + (u-g)/t are produced by one stencil pass (each voxel's q = D u / phi
// computed once and handed to the neighbours that need it; HBM sees u, g in and d out).  Trial
// energies E_R(u - s_m d) for M step sizes s_m = t alpha^m come from one more pass, so one pass
// covers several backtracking steps.
//
// Every reduction is two-level and fixed-order: each work-group of a fixed-size grid writes
// FP64 partial sums, and a single-work-group kernel sums them in order, so results are
// bitwise reproducible and independent of timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

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

// Work distribution of the energy pass: lanes run along x (64 per row segment), work-groups take
// (row segment, 4 rows) tiles and stride over the (y, z) rows, so there is one division per row
// and the grid (hence the partial-sum layout) is fixed by the shape.
struct RowIter {
    int nrow, row0, rstep, a0, astep;
};

// (bx, by) of a (gx, gy) grid: the work-group's place in its volume's grid (the hardware grid of a
// solo launch, a request's share of a batched one)
struct Blk2 {
    int bx, by, gx, gy;
};

__device__ __forceinline__ Blk2 hw_blk2() { return Blk2{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)gridDim.y}; }

__device__ __forceinline__ RowIter row_iter(const TVShape &k, const Blk2 &B) {
    RowIter it;
    it.nrow = k.ny * k.nz;
    it.row0 = B.by * 4 + (threadIdx.x >> 6);
    it.rstep = B.gy * 4;
    it.a0 = B.bx * 64 + (threadIdx.x & 63);
    it.astep = B.gx * 64;
    return it;
}

// ---- per-voxel passes (small volumes: too few tiled work items to fill the GPU) -------------
// Each thread computes its voxel's own and its three lower neighbours' q from u directly.
// d = lambda * N dR/du + (u - g)/t (g may be NULL: then d = N dR/du and lambda is ignored).
// partials[block] = {sum phi, sum (u-g)^2, sum d^2}.
__device__ __forceinline__ void tv_grad_rows(const float *__restrict__ u, const float *__restrict__ g,
                                             float *__restrict__ d, const TVShape &k, float lambda, float inv_t,
                                             double *__restrict__ partials, const Blk2 &B) {
    __shared__ double sh[4];
    const long nxy = (long)k.nx * k.ny;
    double s_phi = 0.0, s_fid = 0.0, s_d2 = 0.0;
    const RowIter ri = row_iter(k, B);
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
    const int blk = B.by * B.gx + B.bx;
    double v;
    v = block_sum(s_phi, sh);
    if (threadIdx.x == 0) partials[blk * 3 + 0] = v;
    v = block_sum(s_fid, sh);
    if (threadIdx.x == 0) partials[blk * 3 + 1] = v;
    v = block_sum(s_d2, sh);
    if (threadIdx.x == 0) partials[blk * 3 + 2] = v;
}

// Trial energies at s_m = s0 * alpha^m, m < M.  partials[block][2m + {0,1}] = {sum phi, sum fid}.
template <int M>
__device__ __forceinline__ void tv_trial_rows(const float *__restrict__ u, const float *__restrict__ d,
                                              const float *__restrict__ g, const TVShape &k, double t, double alpha,
                                              int m0, double *__restrict__ partials, const Blk2 &B) {
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
    const RowIter ri = row_iter(k, B);
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
    const int blk = B.by * B.gx + B.bx;
#pragma unroll
    for (int m = 0; m < M; m++) {
        double v = block_sum(s_phi[m], sh);
        if (threadIdx.x == 0) partials[blk * 2 * M + 2 * m] = v;
        v = block_sum(s_fid[m], sh);
        if (threadIdx.x == 0) partials[blk * 2 * M + 2 * m + 1] = v;
    }
}

// ---- tiled passes: d and the trial energies with the stencil values computed once per voxel ----
// A wave owns a work item: 64 consecutive x (one per lane) x TV_TY rows x zc planes.  It walks
// the item's planes in order and, in every plane, its rows in order, so what a voxel's divergence
// needs from its neighbours is at hand: q_y of the row below from the previous row, q_z of the
// plane below from the previous plane (one register per row), q_x of the voxel to the left from
// lane - 1, u of the row above and of the plane above from the values loaded for them.  The
// item's boundary values are recomputed: the row b0 - 1 in every plane, the plane c0 - 1 for
// every row, and, for lane 0, q_x of the column a0 - 1 over all of the item's rows and planes
// (before the walk, spread over the lanes).  Per voxel, one square root instead of four and two
// loads instead of thirteen.
constexpr int TV_TY = 8;       // rows per work item
constexpr int TV_ZC_MAX = 16;  // planes per work item at most
constexpr int TV_HXR = TV_TY * TV_ZC_MAX / 64;  // registers per lane for the left column's q_x

struct TvItems {
    int tx, ty, tz, zc;  // items along x (64 lanes each), y (TV_TY rows), z (zc planes)
    __host__ __device__ long n() const { return (long)tx * ty * tz; }
};

// items of a volume: enough for about 4096 waves where the volume allows, zc in [4, 16]
static TvItems tv_items(int nx, int ny, int nz) {
    TvItems T;
    T.tx = (nx + 63) / 64;
    T.ty = (ny + TV_TY - 1) / TV_TY;
    const long base = (long)T.tx * T.ty;
    const long chunks = std::max(1L, (4096 + base - 1) / base);
    int zc = (int)((nz + chunks - 1) / chunks);
    zc = std::min(TV_ZC_MAX, std::max(zc, std::min(nz, 4)));
    T.zc = zc;
    T.tz = (nz + zc - 1) / zc;
    return T;
}

// u(a+1, b, c) for every lane: lane + 1's value, and for lane 63 a load (0 outside the grid)
__device__ __forceinline__ float x_next(float v, const float *__restrict__ u, long p, bool inside) {
    float t = __shfl_down(v, 1, 64);
    if ((threadIdx.x & 63) == 63) t = inside ? u[p + 1] : 0.0f;
    return t;
}

// d = lambda N dR/du + (u - g)/t (g NULL: d = N dR/du) over the items w0, w0 + wstep, ...
__device__ __forceinline__ void tv_grad_walk(const float *__restrict__ u, const float *__restrict__ g,
                                             float *__restrict__ d, const TVShape &k, float lambda, float inv_t,
                                             const TvItems &T, int w0, int wstep, double &s_phi, double &s_fid,
                                             double &s_d2) {
    const int lane = threadIdx.x & 63;
    const long nxy = (long)k.nx * k.ny;
    const int nw = (int)T.n();
    for (int w = w0; w < nw; w += wstep) {
        const int ix = w % T.tx, rest = w / T.tx;
        const int iy = rest % T.ty, iz = rest / T.ty;
        const int a = ix * 64 + lane, b0 = iy * TV_TY, c0 = iz * T.zc, c1 = min(k.nz, c0 + T.zc);
        const bool ax = a < k.nx, ax1 = a + 1 < k.nx;
        // u(a, b, c), 0 outside the grid
        const auto ld = [&](int b, int c) -> float {
            return (ax && b >= 0 && b < k.ny) ? u[(long)c * nxy + (long)b * k.nx + a] : 0.0f;
        };
        // u(a+1, b, c) from u(a, b, c) = v, 0 outside the grid
        const auto xn = [&](float v, int b, int c) -> float {
            const bool in = ax1 && b >= 0 && b < k.ny;
            const float t = x_next(v, u, (long)c * nxy + (long)b * k.nx + a, in);
            return in ? t : 0.0f;
        };
        float cu[TV_TY + 2];  // u of rows b0-1 .. b0+TV_TY at the current plane
        float cz[TV_TY];      // q_z of rows b0 .. at the plane below
#pragma unroll
        for (int j = 0; j < TV_TY + 2; j++) cu[j] = ld(b0 - 1 + j, c0);
        if (c0 > 0) {
            float lo[TV_TY + 1];
#pragma unroll
            for (int j = 0; j <= TV_TY; j++) lo[j] = ld(b0 + j, c0 - 1);
#pragma unroll
            for (int j = 0; j < TV_TY; j++) {
                const int b = b0 + j;
                const float v0 = lo[j], vx = xn(v0, b, c0 - 1), vy = (b + 1 < k.ny) ? lo[j + 1] : 0.0f;
                const float dx = (vx - v0) * k.ihx, dy = (vy - v0) * k.ihy, dz = (cu[j + 1] - v0) * k.ihz;
                cz[j] = dz * __builtin_amdgcn_rcpf(phi_of(dx, dy, dz, k.eps2));
            }
        } else {
#pragma unroll
            for (int j = 0; j < TV_TY; j++) cz[j] = 0.0f;
        }
        // q_x of the column a0 - 1 for the item's rows and planes: point i = (c - c0) * TV_TY + (b - b0)
        // in register i / 64 of lane i % 64
        float hx[TV_HXR];
#pragma unroll
        for (int r = 0; r < TV_HXR; r++) {
            hx[r] = 0.0f;
            const int i = lane + 64 * r;
            const int b = b0 + i % TV_TY, c = c0 + i / TV_TY;
            if (ix > 0 && c < c1 && b < k.ny) {
                const long p = (long)c * nxy + (long)b * k.nx + (ix * 64 - 1);
                const float v0 = u[p], vx = u[p + 1];
                const float vy = (b + 1 < k.ny) ? u[p + k.nx] : 0.0f;
                const float vz = (c + 1 < k.nz) ? u[p + nxy] : v0;
                const float dx = (vx - v0) * k.ihx, dy = (vy - v0) * k.ihy, dz = (vz - v0) * k.ihz;
                hx[r] = dx * __builtin_amdgcn_rcpf(phi_of(dx, dy, dz, k.eps2));
            }
        }
        for (int c = c0; c < c1; c++) {
            const bool zin = c + 1 < k.nz;
            float nu[TV_TY + 2];  // u at the plane above (the last plane: its own values, dz = 0)
#pragma unroll
            for (int j = 0; j < TV_TY + 2; j++) nu[j] = zin ? ld(b0 - 1 + j, c + 1) : cu[j];
            float gv[TV_TY];
#pragma unroll
            for (int j = 0; j < TV_TY; j++) {
                const int b = b0 + j;
                gv[j] = (g && ax && b < k.ny) ? g[(long)c * nxy + (long)b * k.nx + a] : 0.0f;
            }
            // q_y of the row below b0 (recomputed: it belongs to the item below)
            float qy_prev = 0.0f;
            if (b0 > 0) {
                const int b = b0 - 1;
                const float v0 = cu[0], vx = xn(v0, b, c), vy = cu[1];
                const float dx = (vx - v0) * k.ihx, dy = (vy - v0) * k.ihy, dz = (nu[0] - v0) * k.ihz;
                qy_prev = dy * __builtin_amdgcn_rcpf(phi_of(dx, dy, dz, k.eps2));
            }
#pragma unroll
            for (int j = 0; j < TV_TY; j++) {
                const int b = b0 + j;
                const float v0 = cu[j + 1], vx = xn(v0, b, c), vy = (b + 1 < k.ny) ? cu[j + 2] : 0.0f;
                const float dx = (vx - v0) * k.ihx, dy = (vy - v0) * k.ihy, dz = (nu[j + 1] - v0) * k.ihz;
                const float ph = phi_of(dx, dy, dz, k.eps2);
                const float ip = __builtin_amdgcn_rcpf(ph);
                const float qx = dx * ip, qy = dy * ip, qz = dz * ip;
                float div = -(qx * k.ihx + qy * k.ihy + qz * k.ihz);
                // q_x of the voxel to the left: lane - 1, or for lane 0 the recomputed column
                float left = __shfl_up(qx, 1, 64);
                const int i = (c - c0) * TV_TY + j;
                float hsrc = hx[0];
#pragma unroll
                for (int r = 1; r < TV_HXR; r++)
                    if ((i >> 6) == r) hsrc = hx[r];
                const float hv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hsrc), i & 63));
                if (lane == 0) left = hv;
                if (a >= 1) div += left * k.ihx;
                if (b >= 1) div += qy_prev * k.ihy;
                if (c >= 1) div += cz[j] * k.ihz;
                qy_prev = qy;
                cz[j] = qz;
                if (ax && b < k.ny) {
                    float dv;
                    if (g) {
                        const float r = v0 - gv[j];
                        dv = fmaf(lambda, div, r * inv_t);
                        s_fid += (double)r * (double)r;
                    } else {
                        dv = div;
                    }
                    d[(long)c * nxy + (long)b * k.nx + a] = dv;
                    s_phi += (double)ph;
                    s_d2 += (double)dv * (double)dv;
                }
            }
#pragma unroll
            for (int j = 0; j < TV_TY + 2; j++) cu[j] = nu[j];
        }
    }
}

// trial energies E_R(u - s_m d), m < M, over the items w0, w0 + wstep, ...: per voxel the forward
// differences of w = u - s_m d from the loaded u and d of the voxel, lane + 1, the row above (loaded
// with the item's rows) and the plane above (loaded for the next plane)
template <int M>
__device__ __forceinline__ void tv_trial_walk(const float *__restrict__ u, const float *__restrict__ d,
                                              const float *__restrict__ g, const TVShape &k, const float *s,
                                              const TvItems &T, int w0, int wstep, double *s_phi, double *s_fid) {
    const int lane = threadIdx.x & 63;
    const long nxy = (long)k.nx * k.ny;
    const int nw = (int)T.n();
    for (int w = w0; w < nw; w += wstep) {
        const int ix = w % T.tx, rest = w / T.tx;
        const int iy = rest % T.ty, iz = rest / T.ty;
        const int a = ix * 64 + lane, b0 = iy * TV_TY, c0 = iz * T.zc, c1 = min(k.nz, c0 + T.zc);
        const bool ax = a < k.nx, ax1 = a + 1 < k.nx;
        const auto ld = [&](const float *__restrict__ v, int b, int c) -> float {
            return (ax && b < k.ny) ? v[(long)c * nxy + (long)b * k.nx + a] : 0.0f;
        };
        const auto xn = [&](const float *__restrict__ v, float val, int b, int c) -> float {
            const bool in = ax1 && b < k.ny;
            const float t = x_next(val, v, (long)c * nxy + (long)b * k.nx + a, in);
            return in ? t : 0.0f;
        };
        float cu[TV_TY + 1], cd[TV_TY + 1];  // rows b0 .. b0+TV_TY at the current plane
#pragma unroll
        for (int j = 0; j <= TV_TY; j++) {
            cu[j] = ld(u, b0 + j, c0);
            cd[j] = ld(d, b0 + j, c0);
        }
        for (int c = c0; c < c1; c++) {
            const bool zin = c + 1 < k.nz;
            float nu[TV_TY + 1], nd[TV_TY + 1];
#pragma unroll
            for (int j = 0; j <= TV_TY; j++) {
                nu[j] = zin ? ld(u, b0 + j, c + 1) : cu[j];
                nd[j] = zin ? ld(d, b0 + j, c + 1) : cd[j];
            }
            float gv[TV_TY];
#pragma unroll
            for (int j = 0; j < TV_TY; j++) gv[j] = ld(g, b0 + j, c);
#pragma unroll
            for (int j = 0; j < TV_TY; j++) {
                const int b = b0 + j;
                const float ux = xn(u, cu[j], b, c), dxv = xn(d, cd[j], b, c);
                const bool yin = b + 1 < k.ny;
                if (ax && b < k.ny) {
#pragma unroll
                    for (int m = 0; m < M; m++) {
                        const float w0v = fmaf(-s[m], cd[j], cu[j]);
                        const float wx = fmaf(-s[m], dxv, ux);
                        const float wy = yin ? fmaf(-s[m], cd[j + 1], cu[j + 1]) : 0.0f;
                        const float wz = fmaf(-s[m], nd[j], nu[j]);
                        const float r = w0v - gv[j];
                        s_phi[m] += (double)phi_of((wx - w0v) * k.ihx, (wy - w0v) * k.ihy, (wz - w0v) * k.ihz,
                                                   k.eps2);
                        s_fid[m] += (double)r * (double)r;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j <= TV_TY; j++) {
                cu[j] = nu[j];
                cd[j] = nd[j];
            }
        }
    }
}

// d = lambda * N dR/du + (u - g)/t (g may be NULL: then d = N dR/du and lambda is ignored) on work
// group blk of nblk (4 waves, 4 items at a time).  partials[blk] = {sum phi, sum (u-g)^2, sum d^2}.
__device__ __forceinline__ void tv_grad_body(const float *__restrict__ u, const float *__restrict__ g,
                                             float *__restrict__ d, const TVShape &k, float lambda, float inv_t,
                                             const TvItems &T, double *__restrict__ partials, int blk, int nblk) {
    __shared__ double sh[4];
    double s_phi = 0.0, s_fid = 0.0, s_d2 = 0.0;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    tv_grad_walk(u, g, d, k, lambda, inv_t, T, blk * 4 + wave, nblk * 4, s_phi, s_fid, s_d2);
    double v;
    v = block_sum(s_phi, sh);
    if (threadIdx.x == 0) partials[blk * 3 + 0] = v;
    v = block_sum(s_fid, sh);
    if (threadIdx.x == 0) partials[blk * 3 + 1] = v;
    v = block_sum(s_d2, sh);
    if (threadIdx.x == 0) partials[blk * 3 + 2] = v;
}

// The layout of a volume's gradient and trial passes: tiled items, or per-voxel rows on a
// (gx, gy) grid of (64-voxel row segment, 4 rows) tiles; nb work-groups in a 1-D launch either way
// (and nb rows of partial sums).
struct TvGrid {
    TvItems T;
    int tiled, gx, gy, nb;
};

__device__ __forceinline__ void tv_grad_any(const float *__restrict__ u, const float *__restrict__ g,
                                            float *__restrict__ d, const TVShape &k, float lambda, float inv_t,
                                            const TvGrid &G, double *__restrict__ partials, int blk) {
    if (G.tiled) tv_grad_body(u, g, d, k, lambda, inv_t, G.T, partials, blk, G.nb);
    else tv_grad_rows(u, g, d, k, lambda, inv_t, partials, Blk2{blk % G.gx, blk / G.gx, G.gx, G.gy});
}

__global__ void __launch_bounds__(256) k_tv_grad(const float *__restrict__ u, const float *__restrict__ g,
                                                 float *__restrict__ d, TVShape k, float lambda, float inv_t,
                                                 TvGrid G, double *__restrict__ partials) {
    tv_grad_any(u, g, d, k, lambda, inv_t, G, partials, blockIdx.x);
}

// sum phi only (energy of a volume)
__global__ void __launch_bounds__(256) k_tv_energy(const float *__restrict__ u, TVShape k,
                                                   double *__restrict__ partials) {
    __shared__ double sh[4];
    const long nxy = (long)k.nx * k.ny;
    double s_phi = 0.0;
    const RowIter ri = row_iter(k, hw_blk2());
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

// Trial energies at s_m = s0 * alpha^m, m < M, on work group blk of nblk.
// partials[blk][2m + {0,1}] = {sum phi, sum fid}.
template <int M>
__device__ __forceinline__ void tv_trial_body(const float *__restrict__ u, const float *__restrict__ d,
                                              const float *__restrict__ g, const TVShape &k, double t, double alpha,
                                              int m0, const TvItems &T, double *__restrict__ partials, int blk,
                                              int nblk) {
    __shared__ double sh[4];
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
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    tv_trial_walk<M>(u, d, g, k, s, T, blk * 4 + wave, nblk * 4, s_phi, s_fid);
#pragma unroll
    for (int m = 0; m < M; m++) {
        double v = block_sum(s_phi[m], sh);
        if (threadIdx.x == 0) partials[blk * 2 * M + 2 * m] = v;
        v = block_sum(s_fid[m], sh);
        if (threadIdx.x == 0) partials[blk * 2 * M + 2 * m + 1] = v;
    }
}

template <int M>
__device__ __forceinline__ void tv_trial_any(const float *__restrict__ u, const float *__restrict__ d,
                                             const float *__restrict__ g, const TVShape &k, double t, double alpha,
                                             int m0, const TvGrid &G, double *__restrict__ partials, int blk) {
    if (G.tiled) tv_trial_body<M>(u, d, g, k, t, alpha, m0, G.T, partials, blk, G.nb);
    else tv_trial_rows<M>(u, d, g, k, t, alpha, m0, partials, Blk2{blk % G.gx, blk / G.gx, G.gx, G.gy});
}

template <int M>
__global__ void __launch_bounds__(256) k_tv_trial(const float *__restrict__ u, const float *__restrict__ d,
                                                  const float *__restrict__ g, TVShape k, double t, double alpha,
                                                  int m0, TvGrid G, double *__restrict__ partials) {
    tv_trial_any<M>(u, d, g, k, t, alpha, m0, G, partials, blockIdx.x);
}

// sum of `nb` rows of `width` partials: out[j] = sum_b part[b * width + j], in a fixed order
// (each thread sums a contiguous run of rows, then a fixed binary tree over the threads), so the
// result does not depend on timing
constexpr int SUM_MAXW = 3 + 2 * CBCT_TRIALS;
__device__ __forceinline__ void sum_rows_body(const double *__restrict__ part, int nb, int width,
                                              double *__restrict__ out) {
    // thread t sums rows t, t + 256, ... (coalesced loads, several in flight), each wave folds its
    // 64 lanes with a fixed butterfly (lane 0's result is kept), and the wave totals are added in
    // wave order: a fixed order, so the sums are bitwise reproducible
    __shared__ double sh[4][SUM_MAXW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double s[SUM_MAXW];
#pragma unroll
    for (int j = 0; j < SUM_MAXW; j++) s[j] = 0.0;
    int b = tid;
    for (; b + 3 * 256 < nb; b += 4 * 256) {
        double v[4][SUM_MAXW];
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int j = 0; j < SUM_MAXW; j++) v[u][j] = j < width ? part[(long)(b + u * 256) * width + j] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int j = 0; j < SUM_MAXW; j++) s[j] += v[u][j];
    }
    for (; b < nb; b += 256) {
#pragma unroll
        for (int j = 0; j < SUM_MAXW; j++)
            if (j < width) s[j] += part[(long)b * width + j];
    }
#pragma unroll
    for (int j = 0; j < SUM_MAXW; j++) {
        double v = s[j];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) sh[wave][j] = v;
    }
    __syncthreads();
    if (tid < width) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) t += sh[w][tid];
        out[tid] = t;
    }
}

__global__ void __launch_bounds__(256) k_sum_rows(const double *__restrict__ part, int nb, int width,
                                                  double *__restrict__ out) {
    sum_rows_body(part, nb, width, out);
}

__device__ __forceinline__ void axpy_step_body(float *__restrict__ u, const float *__restrict__ d,
                                               const RofControl *__restrict__ ctl, long n, int blk, int nblk) {
    if (ctl->accepted != 1) return;
    const float s = (float)ctl->s;
    for (long p = (long)blk * blockDim.x + threadIdx.x; p < n; p += (long)nblk * blockDim.x)
        u[p] = fmaf(-s, d[p], u[p]);
}

__global__ void k_axpy_step(float *__restrict__ u, const float *__restrict__ d, const RofControl *__restrict__ ctl,
                            long n) {
    axpy_step_body(u, d, ctl, n, blockIdx.x, gridDim.x);
}

// Armijo decision for one ROF iteration from the reduced sums.
// sums: [0..2] = {sum phi(u), sum (u-g)^2, sum d^2}, [3 + 2m + {0,1}] = trial sums for m - m0.
// The record goes to ctl (read by the update kernel) and, when given, to a host-mapped mirror
// (no copy command): its fields first, then, after a system-scope fence, the call's sequence
// number in `pad`, so that a host that sees the number also sees the fields.
__device__ __forceinline__ void rof_decide_body(const double *__restrict__ sums, int M, int m0, int forced_m,
                                                double inv_n, double lambda, double t, double c_armijo, double alpha,
                                                int max_bt, RofControl *__restrict__ ctl,
                                                RofControl *__restrict__ mirror, int seq) {
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

__global__ void k_rof_decide(const double *__restrict__ sums, int M, int m0, int forced_m, double inv_n, double lambda,
                             double t, double c_armijo, double alpha, int max_bt, RofControl *__restrict__ ctl,
                             RofControl *__restrict__ mirror, int seq) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    rof_decide_body(sums, M, m0, forced_m, inv_n, lambda, t, c_armijo, alpha, max_bt, ctl, mirror, seq);
}


// ---- Step 2 in one work-group: the whole ROF loop of a small volume on the device ----------
// For volumes of a few tens of thousands of voxels every pass is a few microseconds of work, and
// the loop is bound by launches and by the host reading each Armijo decision.  One work-group of
// 1024 threads runs the whole loop instead: the gradient pass, the backtracking trials (one step
// size per pass, s_m = t alpha^m formed as the multi-kernel path forms it), the decision and the
// update, with work-group barriers between passes and fixed-order FP64 sums, and appends one
// record per ROF iteration.  The per-voxel arithmetic is the multi-kernel path's (same helpers).
constexpr int SMALL_THREADS = 1024;

__device__ double small_block_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < nw; k++) s += sh[k];  // every thread, same order
    return s;
}

__global__ void k_rof_small_init(RofLog *st, int replay_pos) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->n_rec = 0;
        st->replay_pos = replay_pos;
        st->status = 0;
        st->pad = 0;
    }
}

__global__ void __launch_bounds__(SMALL_THREADS)
    k_rof_small(float *__restrict__ u, const float *__restrict__ g, float *__restrict__ d, TVShape k, double lambda,
                double t, double c_armijo, double alpha, double tol, int max_iter, int max_bt,
                const int *__restrict__ replay, int replay_len, RofLog *__restrict__ st,
                RofRecord *__restrict__ rec, int rec_cap, int level, int outer) {
    __shared__ double sh[SMALL_THREADS / 64];
    const long nxy = (long)k.nx * k.ny;
    const int nrow = k.ny * k.nz;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const double inv_n = 1.0 / ((double)nxy * k.nz);
    const float inv_t = (float)(1.0 / t);
    int pos = st->replay_pos;
    int nrec = st->n_rec;
    for (int it = 0; it < max_iter; it++) {
        int forced = -2, fend = -1;
        if (replay && pos < replay_len) {
            forced = replay[2 * pos];
            fend = replay[2 * pos + 1] != 0 ? 1 : 0;
            pos++;
        }
        // gradient pass: d, sum phi, sum (u-g)^2, sum d^2
        double s_phi = 0.0, s_fid = 0.0, s_d2 = 0.0;
        for (int row = wave; row < nrow; row += nw) {
            const int c = row / k.ny, b = row - c * k.ny;
            const long rbase = (long)c * nxy + (long)b * k.nx;
            for (int a = lane; a < k.nx; a += 64) {
                const long p = rbase + a;
                float dx, dy, dz;
                diffs(u, p, a, b, c, k, dx, dy, dz);
                const float ph = phi_of(dx, dy, dz, k.eps2);
                const float ip = __builtin_amdgcn_rcpf(ph);
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
                const float r = u[p] - g[p];
                const float dv = fmaf((float)lambda, div, r * inv_t);
                s_fid += (double)r * (double)r;
                d[p] = dv;
                s_phi += (double)ph;
                s_d2 += (double)dv * (double)dv;
            }
        }
        s_phi = small_block_sum(s_phi, sh);
        s_fid = small_block_sum(s_fid, sh);
        s_d2 = small_block_sum(s_d2, sh);
        const double e0 = lambda * s_phi * inv_n + s_fid * inv_n / (2.0 * t);
        const double G = s_d2 * inv_n;
        // backtracking search, one step size per pass (the forced exponent directly when replaying)
        int m_acc = -1;
        double e_trial = 0.0, s_acc = 0.0;
        if (forced != -1) {
            const int m_first = forced >= 0 ? forced : 0;
            double sd = t;
            for (int m = 0; m < m_first; m++) sd *= alpha;
            for (int m = m_first; m <= max_bt; m++) {
                const float sf = (float)sd;
                double tp = 0.0, tf = 0.0;
                for (int row = wave; row < nrow; row += nw) {
                    const int c = row / k.ny, b = row - c * k.ny;
                    const long rbase = (long)c * nxy + (long)b * k.nx;
                    for (int a = lane; a < k.nx; a += 64) {
                        const long p = rbase + a;
                        float w0, dx, dy, dz;
                        diffs_step(u, d, sf, p, a, b, c, k, w0, dx, dy, dz);
                        const float r = w0 - g[p];
                        tp += (double)phi_of(dx, dy, dz, k.eps2);
                        tf += (double)r * (double)r;
                    }
                }
                tp = small_block_sum(tp, sh);
                tf = small_block_sum(tf, sh);
                e_trial = lambda * tp * inv_n + tf * inv_n / (2.0 * t);
                const bool ok = forced >= 0 ? (m == forced) : (e_trial <= e0 - c_armijo * sd * G);
                if (ok) {
                    m_acc = m;
                    s_acc = sd;
                    break;
                }
                if (forced >= 0) break;
                sd *= alpha;
            }
        }
        if (threadIdx.x == 0 && rec && nrec < rec_cap) {
            RofRecord R;
            R.e0 = e0;
            R.e_trial = e_trial;
            R.G = G;
            R.level = level;
            R.outer = outer;
            R.inner = it;
            R.m = m_acc;
            rec[nrec] = R;
        }
        nrec++;
        if (!isfinite(e0) || !isfinite(G)) {
            if (threadIdx.x == 0) st->status = 1;
            break;
        }
        if (m_acc < 0) break;  // Eq. 5 held for no step: keep u
        const bool own_stop = e0 == 0.0 || G == 0.0 || fabs(e_trial - e0) / e0 < tol;
        const bool stop = (fend >= 0 ? fend == 1 : own_stop) || it + 1 == max_iter;
        const float sf = (float)s_acc;
        __syncthreads();  // every thread has read u for the search
        for (int row = wave; row < nrow; row += nw) {
            const long rbase = (long)row * k.nx;
            for (int a = lane; a < k.nx; a += 64) u[rbase + a] = fmaf(-sf, d[rbase + a], u[rbase + a]);
        }
        __syncthreads();
        if (stop) break;
    }
    if (threadIdx.x == 0) {
        st->n_rec = nrec;
        st->replay_pos = pos;
    }
}


// ---- Step 2 as flag-gated launch chains (larger volumes) -----------------------------------
// The host enqueues whole steps ahead of the decisions: apply the last accepted step, a new
// gradient, one trial window, the decision.  Each kernel reads the loop's state first and returns
// at once when the loop has ended or the step does not need it, so the steps enqueued after the
// loop's last decision cost a few microseconds each, and the device never waits for the host
// between ROF iterations or backtracking windows.  The passes are the multi-kernel path's, and
// the decision kernel forms the sums in k_sum_rows's order and decides with the same body, so the
// results are bitwise those of a host-driven loop over the same kernels.
__global__ void k_axpy_gated(float *__restrict__ u, const float *__restrict__ d, const RofControl *__restrict__ ctl,
                             const RofGate *__restrict__ gate, long n, int pending_only) {
    const bool on = pending_only ? gate->pending != 0 : (gate->run != 0 && gate->apply != 0);
    if (!on) return;
    axpy_step_body(u, d, ctl, n, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) k_tv_grad_gated(const float *__restrict__ u, const float *__restrict__ g,
                                                       float *__restrict__ d, TVShape k, float lambda, float inv_t,
                                                       TvGrid G, double *__restrict__ partials,
                                                       const RofGate *__restrict__ gate) {
    if (!gate->run || !gate->grad) return;
    tv_grad_any(u, g, d, k, lambda, inv_t, G, partials, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_tv_trial_gated(const float *__restrict__ u, const float *__restrict__ d,
                                                        const float *__restrict__ g, TVShape k, double t,
                                                        double alpha, TvGrid G, double *__restrict__ partials,
                                                        const RofGate *__restrict__ gate) {
    if (!gate->run) return;
    const int m0 = gate->m0;
    // the first window tries the full step only, later ones CBCT_TRIALS step sizes
    if (m0 == 0) tv_trial_any<1>(u, d, g, k, t, alpha, 0, G, partials, blockIdx.x);
    else tv_trial_any<CBCT_TRIALS>(u, d, g, k, t, alpha, m0, G, partials, blockIdx.x);
}

struct GateDecide {
    const double *pg, *pt;  // gradient and trial partials
    double *sums;
    int nb;  // rows of gradient and of trial partials
    double inv_n, lambda, t, c_armijo, alpha, tol;
    int max_iter, max_bt;
    RofControl *ctl;
    RofGate *gate;
    RofLog *st;
    const int *replay;
    int replay_len;
    RofRecord *rec;
    int rec_cap, level, outer;
    int *mirror;
    int seq;
    int first;       // the loop's first step: the state starts fresh here (no reset launch)
    int init_state;  // with first: the level's first loop (records and replay position start too)
    int replay_pos;  // with init_state: the replay position at the level's start
};

// the decision of a gated step (one work-group of 256 threads): the fixed-order sums of the step's
// passes, the Armijo decision, the loop's next state, the iteration's record, the host's word
__device__ __forceinline__ void gate_decide_body(const GateDecide &A) {
    __shared__ int run_s, grad_s, m0_s;
    if (threadIdx.x == 0) {
        run_s = A.first ? 1 : A.gate->run;
        grad_s = A.first ? 1 : A.gate->grad;
        m0_s = A.first ? 0 : A.gate->m0;
    }
    __syncthreads();
    if (!run_s) return;
    const int M = m0_s == 0 ? 1 : CBCT_TRIALS;
    if (grad_s) sum_rows_body(A.pg, A.nb, 3, A.sums);
    __syncthreads();
    sum_rows_body(A.pt, A.nb, 2 * M, A.sums + 3);
    __syncthreads();
    if (threadIdx.x != 0) return;
    RofGate G{};
    if (A.first) {
        G.run = 1;
        G.grad = 1;
    } else {
        G = *A.gate;
    }
    RofLog S{};
    if (A.first && A.init_state) S.replay_pos = A.replay_pos;
    else S = *A.st;
    // the replayed decision of this ROF iteration, if any (applies to all of its windows)
    int forced = -2, fend = -1;
    if (A.replay && S.replay_pos < A.replay_len) {
        forced = A.replay[2 * S.replay_pos];
        fend = A.replay[2 * S.replay_pos + 1] != 0 ? 1 : 0;
    }
    RofControl c{};
    if (forced == -1) {
        // replayed: the search found no admissible step (the iteration's gradient sums only)
        c.e0 = A.lambda * A.sums[0] * A.inv_n + A.sums[1] * A.inv_n / (2.0 * A.t);
        c.G = A.sums[2] * A.inv_n;
        c.accepted = -1;
        *A.ctl = c;
    } else {
        rof_decide_body(A.sums, M, m0_s, forced, A.inv_n, A.lambda, A.t, A.c_armijo, A.alpha, A.max_bt, A.ctl,
                        nullptr, 0);
        c = *A.ctl;
    }
    if (c.accepted == 0 && c.next_m0 > m0_s) {
        // the next window, same gradient
        G.m0 = c.next_m0;
        G.apply = 0;
        G.grad = 0;
    } else {
        if (forced != -2) S.replay_pos++;
        if (A.rec && S.n_rec < A.rec_cap) {
            RofRecord R;
            R.e0 = c.e0;
            R.e_trial = c.e_trial;
            R.G = c.G;
            R.level = A.level;
            R.outer = A.outer;
            R.inner = G.it;
            R.m = c.accepted == 1 ? c.m : -1;
            A.rec[S.n_rec] = R;
        }
        S.n_rec++;
        if (!isfinite(c.e0) || !isfinite(c.G)) {
            S.status = 1;
            G.run = 0;
        } else if (c.accepted != 1) {
            G.run = 0;  // Eq. 5 held for no step: keep u
        } else {
            const bool own_stop =
                c.e0 == 0.0 || c.G == 0.0 || fabs(c.e_trial - c.e0) / c.e0 < A.tol;
            const bool stop = (fend >= 0 ? fend == 1 : own_stop) || G.it + 1 == A.max_iter;
            if (stop) {
                G.run = 0;
                G.pending = 1;
            } else {
                G.apply = 1;
                G.grad = 1;
                G.m0 = 0;
                G.it++;
            }
        }
    }
    *A.gate = G;
    *A.st = S;
    if (A.mirror) {
        __threadfence_system();
        *reinterpret_cast<volatile int *>(A.mirror) = cbct_gate_word(A.seq, S.status, G.run);
    }
}

__global__ void __launch_bounds__(256) k_rof_decide_gated(GateDecide A) { gate_decide_body(A); }

// ---- batched kernels (serving engine) ------------------------------------------------------
// One gated step of several requests' Step 2 in shared launches: each request's work-groups run
// the solo kernels' bodies on its buffers, grid and loop state (so its results are bitwise its
// solo results), and a request whose loop has ended leaves its work-groups idle.
struct BStepItem {
    float *u;
    const float *g;
    float *d;
    double *pg, *pt;  // gradient and trial partials
    const RofControl *ctl;
    const RofGate *gate;
    TVShape k;
    float lambda, inv_t;
    double t, alpha;
    TvGrid G;     // layout of its gradient and trial passes (nb: their work-groups)
    long n;
    int nba;      // its update work-groups
};
struct BStep {
    int n;
    int first;               // the loops' first step: the passes run without reading any state
    int wg0[CBCT_MAXB + 1];  // exclusive prefix of the TV passes' work-groups
    int wa0[CBCT_MAXB + 1];  // the same for the update pass
    BStepItem it[CBCT_MAXB];
};

// the request a work-group of a batched launch belongs to (wg0: exclusive prefix of work-groups)
__device__ __forceinline__ int batch_of(const int *wg0, int n, int w) {
    int r = 0;
    while (r + 1 < n && w >= wg0[r + 1]) r++;
    return r;
}

__global__ void k_axpy_gated_b(BStep B) {
    const int r = batch_of(B.wa0, B.n, blockIdx.x);
    const BStepItem &it = B.it[r];
    if (!it.gate->run || !it.gate->apply) return;
    axpy_step_body(it.u, it.d, it.ctl, it.n, blockIdx.x - B.wa0[r], it.nba);
}

__global__ void __launch_bounds__(256) k_tv_grad_gated_b(BStep B) {
    const int r = batch_of(B.wg0, B.n, blockIdx.x);
    const BStepItem &it = B.it[r];
    if (!B.first && (!it.gate->run || !it.gate->grad)) return;
    tv_grad_any(it.u, it.g, it.d, it.k, it.lambda, it.inv_t, it.G, it.pg, blockIdx.x - B.wg0[r]);
}

__global__ void __launch_bounds__(256) k_tv_trial_gated_b(BStep B) {
    const int r = batch_of(B.wg0, B.n, blockIdx.x);
    const BStepItem &it = B.it[r];
    if (!B.first && !it.gate->run) return;
    const int m0 = B.first ? 0 : it.gate->m0, local = blockIdx.x - B.wg0[r];
    if (m0 == 0) tv_trial_any<1>(it.u, it.d, it.g, it.k, it.t, it.alpha, 0, it.G, it.pt, local);
    else tv_trial_any<CBCT_TRIALS>(it.u, it.d, it.g, it.k, it.t, it.alpha, m0, it.G, it.pt, local);
}

struct BDecide {
    int n;
    GateDecide it[CBCT_MAXB];
};
// kernel arguments are at most 4 KB
static_assert(sizeof(BStep) <= 4096 && sizeof(BDecide) <= 4096, "batched step arguments");

// one work-group per request
__global__ void __launch_bounds__(256) k_rof_decide_gated_b(BDecide B) { gate_decide_body(B.it[blockIdx.x]); }

}  // namespace

// ---- launchers ---------------------------------------------------------------------------
static TVShape tv_shape(const Level &L, double eps) {
    return TVShape{L.nx, L.ny, L.nz, (float)(1.0 / L.hx), (float)(1.0 / L.hy), (float)(1.0 / L.hz),
                   (float)(eps * eps)};
}

// grid of the energy pass: (x segments of 64) x (row groups of 4), about CBCT_RED_BLOCKS
// work-groups
static dim3 tv_grid(const Level &L) {
    const int gx = (L.nx + 63) / 64;
    const int rows = (L.ny * L.nz + 3) / 4;
    const int gy = std::max(1, std::min(rows, CBCT_RED_BLOCKS / gx));
    return dim3(gx, gy);
}

// work-groups of the tiled gradient and trial passes (4 items at a time; fixed by the shape, so
// the partial-sum layout is too)
static int tv_blocks(const TvItems &T) {
    return (int)std::min<long>((T.n() + 3) / 4, CBCT_RED_BLOCKS);
}

// the tiled walk where the volume gives at least 1024 items (4096 at 512x512x64, 1024 at 128^3),
// the per-voxel passes below that (a 32^3 volume makes 32 items: eight work-groups walking their
// items serially, against 256 work-groups of independent voxels)
static TvGrid tv_layout(const Level &L) {
    TvGrid G{};
    G.T = tv_items(L.nx, L.ny, L.nz);
    G.tiled = G.T.n() >= 1024;
    if (G.tiled) {
        G.nb = tv_blocks(G.T);
    } else {
        const dim3 g = tv_grid(L);
        G.gx = (int)g.x;
        G.gy = (int)g.y;
        G.nb = G.gx * G.gy;
    }
    return G;
}

int cbct_reduce_blocks(const Level &L) {
    const dim3 g = tv_grid(L);
    return std::max((int)(g.x * g.y), tv_layout(L).nb);
}

#define LAUNCH_CHECK(what)                                  \
    do {                                                    \
        hipError_t e_ = hipGetLastError();                  \
        if (e_ != hipSuccess) return cbct_hip_error(e_, what); \
    } while (0)

cbct_status cbct_launch_tv_grad(const Level &L, double eps, const float *u, const float *g, float *d, double lambda,
                                double t, double *partials, double *sums, hipStream_t s) {
    const TvGrid G = tv_layout(L);
    const int nb = G.nb;
    hipLaunchKernelGGL(k_tv_grad, dim3(nb), dim3(256), 0, s, u, g, d, tv_shape(L, eps), (float)lambda,
                       (float)(1.0 / t), G, partials);
    LAUNCH_CHECK("k_tv_grad");
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, partials, nb, 3, sums);
    LAUNCH_CHECK("k_sum_rows");
    return CBCT_OK;
}

cbct_status cbct_launch_tv_energy(const Level &L, double eps, const float *u, double *partials, double *sum,
                                  hipStream_t s) {
    const dim3 gr = tv_grid(L);
    const int nb = (int)(gr.x * gr.y);
    hipLaunchKernelGGL(k_tv_energy, gr, dim3(256), 0, s, u, tv_shape(L, eps), partials);
    LAUNCH_CHECK("k_tv_energy");
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, partials, nb, 1, sum);
    LAUNCH_CHECK("k_sum_rows");
    return CBCT_OK;
}

cbct_status cbct_launch_tv_trial(const Level &L, double eps, const float *u, const float *d, const float *g,
                                 double t, double alpha, int m0, int M, double *partials, double *sums, hipStream_t s) {
    const TvGrid G = tv_layout(L);
    const int nb = G.nb;
    if (M == 1)
        hipLaunchKernelGGL((k_tv_trial<1>), dim3(nb), dim3(256), 0, s, u, d, g, tv_shape(L, eps), t, alpha, m0, G,
                           partials);
    else
        hipLaunchKernelGGL((k_tv_trial<CBCT_TRIALS>), dim3(nb), dim3(256), 0, s, u, d, g, tv_shape(L, eps), t,
                           alpha, m0, G, partials);
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

cbct_status cbct_launch_rof_small(const Level &L, double eps, float *u, const float *g, float *d, double lambda,
                                  double t, double c_armijo, double alpha, double tol, int max_iter, int max_bt,
                                  const int *replay, int replay_len, int replay_pos, RofLog *st,
                                  RofRecord *rec, int rec_cap, int level, int outer, bool init, hipStream_t s) {
    if (init) {
        hipLaunchKernelGGL(k_rof_small_init, dim3(1), dim3(64), 0, s, st, replay_pos);
        LAUNCH_CHECK("k_rof_small_init");
    }
    hipLaunchKernelGGL(k_rof_small, dim3(1), dim3(SMALL_THREADS), 0, s, u, g, d, tv_shape(L, eps), lambda, t, c_armijo,
                       alpha, tol, max_iter, max_bt, replay, replay_len, st, rec, rec_cap, level, outer);
    LAUNCH_CHECK("k_rof_small");
    return CBCT_OK;
}

static GateDecide gate_decide_args(const Level &L, const RofStepArgs &a, int nb) {
    GateDecide D;
    D.pg = a.part;
    D.pt = a.part + 3 * (size_t)CBCT_RED_BLOCKS;
    D.sums = a.sums;
    D.nb = nb;
    D.inv_n = 1.0 / (double)L.nvox();
    D.lambda = a.lambda;
    D.t = a.t;
    D.c_armijo = a.c_armijo;
    D.alpha = a.alpha;
    D.tol = a.tol;
    D.max_iter = a.max_iter;
    D.max_bt = a.max_bt;
    D.ctl = a.ctl;
    D.gate = a.gate;
    D.st = a.st;
    D.replay = a.replay;
    D.replay_len = a.replay_len;
    D.rec = a.rec;
    D.rec_cap = a.rec_cap;
    D.level = a.level;
    D.outer = a.outer;
    D.mirror = a.mirror;
    D.seq = a.seq & CBCT_GATE_SEQ_MASK;
    D.first = a.first;
    D.init_state = a.init_state;
    D.replay_pos = a.replay_pos;
    return D;
}

cbct_status cbct_launch_rof_step_gated(const Level &L, const RofStepArgs &a, hipStream_t s) {
    const long n = L.nvox();
    const int nba = (int)std::min<long>((n + 255) / 256, 4096);
    const TvGrid G = tv_layout(L);
    const TVShape k = tv_shape(L, a.eps);
    double *pt = a.part + 3 * (size_t)CBCT_RED_BLOCKS;
    if (a.first) {
        // the loop's first step always runs a gradient and the full-step trial: the passes need
        // no state, and the decision starts the state (no reset launch)
        hipLaunchKernelGGL(k_tv_grad, dim3(G.nb), dim3(256), 0, s, a.u, a.g, a.d, k, (float)a.lambda,
                           (float)(1.0 / a.t), G, a.part);
        LAUNCH_CHECK("k_tv_grad");
        hipLaunchKernelGGL((k_tv_trial<1>), dim3(G.nb), dim3(256), 0, s, a.u, a.d, a.g, k, a.t, a.alpha, 0, G,
                           pt);
        LAUNCH_CHECK("k_tv_trial");
    } else {
        hipLaunchKernelGGL(k_axpy_gated, dim3(nba), dim3(256), 0, s, a.u, a.d, a.ctl, a.gate, n, 0);
        LAUNCH_CHECK("k_axpy_gated");
        hipLaunchKernelGGL(k_tv_grad_gated, dim3(G.nb), dim3(256), 0, s, a.u, a.g, a.d, k, (float)a.lambda,
                           (float)(1.0 / a.t), G, a.part, a.gate);
        LAUNCH_CHECK("k_tv_grad_gated");
        hipLaunchKernelGGL(k_tv_trial_gated, dim3(G.nb), dim3(256), 0, s, a.u, a.d, a.g, k, a.t, a.alpha, G, pt,
                           a.gate);
        LAUNCH_CHECK("k_tv_trial_gated");
    }
    const GateDecide D = gate_decide_args(L, a, G.nb);
    hipLaunchKernelGGL(k_rof_decide_gated, dim3(1), dim3(256), 0, s, D);
    LAUNCH_CHECK("k_rof_decide_gated");
    return CBCT_OK;
}

cbct_status cbct_launch_axpy_pending(float *u, const float *d, const RofControl *ctl, const RofGate *gate, long n,
                                     hipStream_t s) {
    const int nb = (int)std::min<long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_axpy_gated, dim3(nb), dim3(256), 0, s, u, d, ctl, gate, n, 1);
    LAUNCH_CHECK("k_axpy_gated");
    return CBCT_OK;
}

// ---- batched launchers ---------------------------------------------------------------------
cbct_status cbct_launch_rof_step_gated_batch(const Level *const *L, const RofStepArgs *a, int n, hipStream_t s) {
    for (int q0 = 0; q0 < n; q0 += CBCT_MAXB) {
        const int m = std::min(CBCT_MAXB, n - q0);
        BStep B{};
        BDecide D{};
        B.n = D.n = m;
        B.first = a[q0].first;  // the steps of one batch are all first steps or none is
        int w = 0, wa = 0;
        for (int q = 0; q < m; q++) {
            const Level &Lq = *L[q0 + q];
            const RofStepArgs &aq = a[q0 + q];
            BStepItem &it = B.it[q];
            it.u = aq.u;
            it.g = aq.g;
            it.d = aq.d;
            it.pg = aq.part;
            it.pt = aq.part + 3 * (size_t)CBCT_RED_BLOCKS;
            it.ctl = aq.ctl;
            it.gate = aq.gate;
            it.k = tv_shape(Lq, aq.eps);
            it.lambda = (float)aq.lambda;
            it.inv_t = (float)(1.0 / aq.t);
            it.t = aq.t;
            it.alpha = aq.alpha;
            it.G = tv_layout(Lq);
            it.n = Lq.nvox();
            it.nba = (int)std::min<long>((it.n + 255) / 256, 4096);
            B.wg0[q] = w;
            B.wa0[q] = wa;
            w += it.G.nb;
            wa += it.nba;
            D.it[q] = gate_decide_args(Lq, aq, it.G.nb);
        }
        B.wg0[m] = w;
        B.wa0[m] = wa;
        if (!B.first) {
            hipLaunchKernelGGL(k_axpy_gated_b, dim3(wa), dim3(256), 0, s, B);
            LAUNCH_CHECK("k_axpy_gated_b");
        }
        hipLaunchKernelGGL(k_tv_grad_gated_b, dim3(w), dim3(256), 0, s, B);
        LAUNCH_CHECK("k_tv_grad_gated_b");
        hipLaunchKernelGGL(k_tv_trial_gated_b, dim3(w), dim3(256), 0, s, B);
        LAUNCH_CHECK("k_tv_trial_gated_b");
        hipLaunchKernelGGL(k_rof_decide_gated_b, dim3(m), dim3(256), 0, s, D);
        LAUNCH_CHECK("k_rof_decide_gated_b");
    }
    return CBCT_OK;
}

// ---- scratch of the no-allocation TV energy / gradient entry point --------------------------
// The fixed-order partial sums of the gradient pass (3 doubles per work-group of the reduction
// grid) and the final sums live in this file-scope device array instead of a caller workspace.
// Each device holds its own copy until the process ends; host code uses the address that
// hipGetSymbolAddress returns for the current device, never the array's name.
static __device__ __align__(256) unsigned char scratch[CBCT_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[CBCT_MAX_DEVICES];

cbct_status cbct_noalloc_scratch_init(int device) {
    if (device < 0 || device >= CBCT_MAX_DEVICES)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "scratch: device %d beyond %d", device, CBCT_MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return CBCT_OK;
    int cur = -1;
    CBCT_HIP(hipGetDevice(&cur));
    if (cur != device) return cbct_set_error(CBCT_ERR_INTERNAL, "scratch: device %d is not current", device);
    void *p = nullptr;
    CBCT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = p;
    return CBCT_OK;
}

void *cbct_noalloc_scratch(int device) {
    if (device < 0 || device >= CBCT_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}
