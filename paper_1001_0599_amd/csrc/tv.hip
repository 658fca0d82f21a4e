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

// Work distribution of the TV kernels: lanes run along x (64 per row segment), work-groups take
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

// d = lambda * N dR/du + (u - g)/t (g may be NULL: then d = N dR/du and lambda is ignored).
// partials[block] = {sum phi, sum (u-g)^2, sum d^2}.
__device__ __forceinline__ void tv_grad_body(const float *__restrict__ u, const float *__restrict__ g,
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

__global__ void __launch_bounds__(256) k_tv_grad(const float *__restrict__ u, const float *__restrict__ g,
                                                 float *__restrict__ d, TVShape k, float lambda, float inv_t,
                                                 double *__restrict__ partials) {
    tv_grad_body(u, g, d, k, lambda, inv_t, partials, hw_blk2());
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

// Trial energies at s_m = s0 * alpha^m, m < M.  partials[block][2m + {0,1}] = {sum phi, sum fid}.
template <int M>
__device__ __forceinline__ void tv_trial_body(const float *__restrict__ u, const float *__restrict__ d,
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

template <int M>
__global__ void __launch_bounds__(256) k_tv_trial(const float *__restrict__ u, const float *__restrict__ d,
                                                  const float *__restrict__ g, TVShape k, double t, double alpha,
                                                  int m0, double *__restrict__ partials) {
    tv_trial_body<M>(u, d, g, k, t, alpha, m0, partials, hw_blk2());
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

__global__ void k_rof_small_init(RofSmallState *st, int replay_pos) {
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
                const int *__restrict__ replay, int replay_len, RofSmallState *__restrict__ st,
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


// ---- batched kernels (serving engine) ------------------------------------------------------
struct BTvItem {
    const float *u, *g;
    float *d;
    double *partials, *out;
    TVShape k;
    float lambda, inv_t;
    double t, alpha;
    int m0, gx, gy;
};
struct BTv {
    int n;
    int wg0[CBCT_MAXB + 1];
    BTvItem it[CBCT_MAXB];
};

// the request a work-group of a batched launch belongs to (wg0: exclusive prefix of work-groups)
__device__ __forceinline__ int batch_of(const int *wg0, int n, int w) {
    int r = 0;
    while (r + 1 < n && w >= wg0[r + 1]) r++;
    return r;
}

__global__ void __launch_bounds__(256) k_tv_grad_b(BTv B) {
    const int r = batch_of(B.wg0, B.n, blockIdx.x);
    const BTvItem &it = B.it[r];
    const int local = blockIdx.x - B.wg0[r];
    tv_grad_body(it.u, it.g, it.d, it.k, it.lambda, it.inv_t, it.partials,
                 Blk2{local % it.gx, local / it.gx, it.gx, it.gy});
}

template <int M>
__global__ void __launch_bounds__(256) k_tv_trial_b(BTv B) {
    const int r = batch_of(B.wg0, B.n, blockIdx.x);
    const BTvItem &it = B.it[r];
    const int local = blockIdx.x - B.wg0[r];
    tv_trial_body<M>(it.u, it.d, it.g, it.k, it.t, it.alpha, it.m0, it.partials,
                     Blk2{local % it.gx, local / it.gx, it.gx, it.gy});
}

// one work-group per request
__global__ void __launch_bounds__(256) k_sum_rows_b(BTv B, int width) {
    const BTvItem &it = B.it[blockIdx.x];
    sum_rows_body(it.partials, it.gx * it.gy, width, it.out);
}

struct BDecItem {
    const double *sums;
    int m0, M, max_bt, seq;
    double inv_n, lambda, t, c_armijo, alpha;
    RofControl *ctl, *mirror;
};
struct BDec {
    int n;
    BDecItem it[CBCT_MAXB];
};

__global__ void k_rof_decide_b(BDec B) {
    const int r = threadIdx.x;
    if (blockIdx.x != 0 || r >= B.n) return;
    const BDecItem &it = B.it[r];
    rof_decide_body(it.sums, it.M, it.m0, -1, it.inv_n, it.lambda, it.t, it.c_armijo, it.alpha, it.max_bt, it.ctl,
                    it.mirror, it.seq);
}

struct BAxItem {
    float *u;
    const float *d;
    const RofControl *ctl;
    long n;
    int nb;
};
struct BAx {
    int n;
    int wg0[CBCT_MAXB + 1];
    BAxItem it[CBCT_MAXB];
};

__global__ void k_axpy_b(BAx B) {
    const int r = batch_of(B.wg0, B.n, blockIdx.x);
    const BAxItem &it = B.it[r];
    axpy_step_body(it.u, it.d, it.ctl, it.n, blockIdx.x - B.wg0[r], it.nb);
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

cbct_status cbct_launch_rof_small(const Level &L, double eps, float *u, const float *g, float *d, double lambda,
                                  double t, double c_armijo, double alpha, double tol, int max_iter, int max_bt,
                                  const int *replay, int replay_len, int replay_pos, RofSmallState *st,
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

// ---- batched launchers ---------------------------------------------------------------------
static BTv make_btv(const TvReq *r, int n, int sums_off) {
    BTv B{};
    B.n = n;
    int w = 0;
    for (int q = 0; q < n; q++) {
        const Level &L = *r[q].L;
        const dim3 gr = tv_grid(L);
        BTvItem &it = B.it[q];
        it.u = r[q].u;
        it.g = r[q].g;
        it.d = r[q].d;
        it.partials = r[q].partials;
        it.out = r[q].sums + sums_off;
        it.k = tv_shape(L, r[q].eps);
        it.lambda = (float)r[q].lambda;
        it.inv_t = (float)(1.0 / r[q].t);
        it.t = r[q].t;
        it.alpha = r[q].alpha;
        it.m0 = r[q].m0;
        it.gx = (int)gr.x;
        it.gy = (int)gr.y;
        B.wg0[q] = w;
        w += it.gx * it.gy;
    }
    B.wg0[n] = w;
    return B;
}

cbct_status cbct_launch_tv_grad_batch(const TvReq *r, int n, hipStream_t s) {
    for (int q0 = 0; q0 < n; q0 += CBCT_MAXB) {
        const int m = std::min(CBCT_MAXB, n - q0);
        const BTv B = make_btv(r + q0, m, 0);
        hipLaunchKernelGGL(k_tv_grad_b, dim3(B.wg0[m]), dim3(256), 0, s, B);
        LAUNCH_CHECK("k_tv_grad_b");
        hipLaunchKernelGGL(k_sum_rows_b, dim3(m), dim3(256), 0, s, B, 3);
        LAUNCH_CHECK("k_sum_rows_b");
    }
    return CBCT_OK;
}

cbct_status cbct_launch_tv_trial_batch(const TvReq *r, int n, int M, hipStream_t s) {
    if (M != 1 && M != CBCT_TRIALS) return cbct_set_error(CBCT_ERR_INTERNAL, "tv_trial_batch: M = %d", M);
    for (int q0 = 0; q0 < n; q0 += CBCT_MAXB) {
        const int m = std::min(CBCT_MAXB, n - q0);
        const BTv B = make_btv(r + q0, m, 3);
        if (M == 1) hipLaunchKernelGGL((k_tv_trial_b<1>), dim3(B.wg0[m]), dim3(256), 0, s, B);
        else hipLaunchKernelGGL((k_tv_trial_b<CBCT_TRIALS>), dim3(B.wg0[m]), dim3(256), 0, s, B);
        LAUNCH_CHECK("k_tv_trial_b");
        hipLaunchKernelGGL(k_sum_rows_b, dim3(m), dim3(256), 0, s, B, 2 * M);
        LAUNCH_CHECK("k_sum_rows_b");
    }
    return CBCT_OK;
}

cbct_status cbct_launch_rof_decide_batch(const DecideReq *r, int n, hipStream_t s) {
    for (int q0 = 0; q0 < n; q0 += CBCT_MAXB) {
        const int m = std::min(CBCT_MAXB, n - q0);
        BDec B{};
        B.n = m;
        for (int q = 0; q < m; q++) {
            const DecideReq &d = r[q0 + q];
            B.it[q] = BDecItem{d.sums, d.m0, d.M, d.max_bt, d.seq, 1.0 / (double)d.nvox, d.lambda, d.t,
                               d.c_armijo, d.alpha, d.ctl, d.mirror};
        }
        hipLaunchKernelGGL(k_rof_decide_b, dim3(1), dim3(64), 0, s, B);
        LAUNCH_CHECK("k_rof_decide_b");
    }
    return CBCT_OK;
}

cbct_status cbct_launch_axpy_batch(const AxpyReq *r, int n, hipStream_t s) {
    for (int q0 = 0; q0 < n; q0 += CBCT_MAXB) {
        const int m = std::min(CBCT_MAXB, n - q0);
        BAx B{};
        B.n = m;
        int w = 0;
        for (int q = 0; q < m; q++) {
            const AxpyReq &a = r[q0 + q];
            const int nb = (int)std::min<long>((a.n + 255) / 256, 4096);
            B.it[q] = BAxItem{a.u, a.d, a.ctl, a.n, nb};
            B.wg0[q] = w;
            w += nb;
        }
        B.wg0[m] = w;
        hipLaunchKernelGGL(k_axpy_b, dim3(w), dim3(256), 0, s, B);
        LAUNCH_CHECK("k_axpy_b");
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
