// Siddon's exact radiological path (the ray tracer of Section II.C.2, also the paper's data
// simulator in Section III.A) as a projector pair: every voxel is constant on its cube and a ray's
// value is the sum over voxels of (length of the ray inside the cube) x (voxel value).
//
// Parameterisation.  All rays of one detector column lie in one vertical plane and share its
// transverse (xy) line.  tau is the transverse distance along that line from C, the line's closest
// approach to the rotation axis (|tau| stays within the grid's half diagonal, so float crossing
// parameters are accurate to ~1e-5 mm; the z crossings, which involve the source distance, are
// formed in FP64 first); the source sits at tau = -t0, the detector at lxy - t0.
// The ray of detector height v has z(tau) = (tau + t0) v / lxy and 3-D length per unit tau of
// sqrt(1 + (v / lxy)^2).  Cubes are half-open on their upper faces (a ray lying in a face plane
// belongs to the cube above it).
//
// Forward: one wave per (view, column, 64 rows).  The xy traversal (which voxel column, the tau
// where the line leaves it) is the same for the whole wave; each lane walks its own z cells inside
// every xy piece, reading the volume in the column-major layout [ny][nx][nz] so that the rows of a
// wave read neighbouring z of one voxel column.
//
// Transpose: a voxel-driven gather with no atomics.  A thread owns SID_TZ cells of one voxel
// column; per view it takes the detector columns whose plane crosses the column's square (from the
// fan projection of its corners), the tau interval of the square on each column's line, and per
// cell the rows whose z range over that interval meets the cell.  Every interval bound is the
// same float expression the forward kernel uses for the corresponding plane crossing, so the pair
// is a transpose up to the order of the sums.
#include "cbct_internal.h"

namespace {

constexpr float SID_INF = __builtin_huge_valf();
constexpr int SID_TZ = 8;  // z cells per thread of the gather

struct SidArgs {
    int nx, ny, nz, nu, nv, nviews;
    float hx, hy, hz, pu, pv, sad, sdd;
    double hzd, pvd;  // hz and pv in FP64 (the z crossings)
};

// plane p (0 .. n) of an axis with n cells of pitch h centred on the origin
__device__ __forceinline__ float sid_plane(int p, int n, float h) { return ((float)p - 0.5f * (float)n) * h; }

// cell of coordinate x on that axis (half-open cells; may lie outside 0 .. n-1)
__device__ __forceinline__ int sid_cell(float x, int n, float h) { return (int)floorf(x / h + 0.5f * (float)n); }

// narrows [lo, hi) to the part of the column's line between planes p0 < p1 of one transverse axis;
// c is the line's coordinate at tau = 0 and ie 1/(its direction component), 0 when the line runs
// parallel to the planes
__device__ __forceinline__ void sid_slab(float c, float ie, int p0, int p1, int n, float h, float &lo, float &hi) {
    if (ie != 0.0f) {
        const float t0 = (sid_plane(p0, n, h) - c) * ie, t1 = (sid_plane(p1, n, h) - c) * ie;
        lo = fmaxf(lo, fminf(t0, t1));
        hi = fminf(hi, fmaxf(t0, t1));
    } else {
        const int k = sid_cell(c, n, h);
        if (k < p0 || k >= p1) hi = -SID_INF;
    }
}

// detector height of row j
__device__ __forceinline__ float sid_row_v(int j, const SidArgs &A) { return ((float)j - 0.5f * (float)(A.nv - 1)) * A.pv; }

// z crossings in FP64.  The ray of detector height v rises v / lxy per unit of tau from the source
// at tau = -t0, so it crosses z plane p at tau = z_p lxy / v - t0.  With t0 (about 1e3 mm) and
// lxy taken from the table's float pairs and z_p, v in FP64, that tau is exact up to its one
// rounding to float (|tau| stays within the grid's half diagonal: ~1e-5 mm), where float
// arithmetic left ~1e-4 mm (the 6e-8 relative error of lxy / v carried over the source
// distance).  Forward and transpose kernels use these same expressions.
__device__ __forceinline__ double sid_t0(const SidCol &c) { return (double)c.t0 + (double)c.t0lo; }

// lxy / v of row j (0 for v = 0: the ray stays in one z cell)
__device__ __forceinline__ double sid_ikz(const SidCol &c, const SidArgs &A, int j) {
    const double v = ((double)j - 0.5 * (double)(A.nv - 1)) * A.pvd;
    return v != 0.0 ? ((double)c.lxy + (double)c.lxylo) / v : 0.0;
}

// tau at which the ray with lxy / v = ikz crosses z plane p
__device__ __forceinline__ float sid_zcross(int p, const SidArgs &A, double ikz, double t0) {
    return (float)fma(((double)p - 0.5 * (double)A.nz) * A.hzd, ikz, -t0);
}

// tau of the next z crossing of a lane in cell cz moving by sz (+-1, 0): none once it has left the grid
__device__ __forceinline__ float sid_znext(int cz, int sz, const SidArgs &A, double ikz, double t0) {
    if (sz > 0) return cz < A.nz ? sid_zcross(cz + 1, A, ikz, t0) : SID_INF;
    if (sz < 0) return cz >= 0 ? sid_zcross(cz, A, ikz, t0) : SID_INF;
    return SID_INF;
}

// z cell of that ray at tau, clamped to [-1, nz] (v = 0: the cell of z = 0)
__device__ __forceinline__ int sid_zcell(float tau, const SidArgs &A, double ikz, double t0) {
    const double z = ikz != 0.0 ? ((double)tau + t0) / ikz : 0.0;
    return (int)fmin(fmax(floor(z / A.hzd + 0.5 * (double)A.nz), -1.0), (double)A.nz);
}

__global__ void __launch_bounds__(256) k_siddon_forward(const float *__restrict__ vol_t, const SidCol *__restrict__ cols,
                                                        SidArgs A, int nchunk, float *__restrict__ out) {
    const int wg = cbct_xcd_remap(blockIdx.x, gridDim.x);
    const long item = (long)wg * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (item >= (long)A.nviews * A.nu * nchunk) return;
    const long vc = item / nchunk;  // view * nu + column
    const int j = (int)(item - vc * nchunk) * 64 + (int)(threadIdx.x & 63);
    const SidCol c = cols[vc];
    const float v = sid_row_v(j, A);
    const float kz = v * c.ilxy;
    float tin = -c.t0, tout = c.lxy - c.t0;
    sid_slab(c.cx, c.iex, 0, A.nx, A.nx, A.hx, tin, tout);
    sid_slab(c.cy, c.iey, 0, A.ny, A.ny, A.hy, tin, tout);
    float acc = 0.0f;
    if (tin < tout) {
        // transverse state, uniform over the wave: voxel column (a, b), its exit parameters
        int a = min(max(sid_cell(fmaf(tin, c.ex, c.cx), A.nx, A.hx), 0), A.nx - 1);
        int b = min(max(sid_cell(fmaf(tin, c.ey, c.cy), A.ny, A.hy), 0), A.ny - 1);
        if (c.iex == 0.0f) a = sid_cell(c.cx, A.nx, A.hx);
        if (c.iey == 0.0f) b = sid_cell(c.cy, A.ny, A.hy);
        const int sx = c.ex > 0.0f ? 1 : -1, sy = c.ey > 0.0f ? 1 : -1;
        float txn = c.iex != 0.0f ? (sid_plane(a + (sx > 0), A.nx, A.hx) - c.cx) * c.iex : SID_INF;
        float tyn = c.iey != 0.0f ? (sid_plane(b + (sy > 0), A.ny, A.hy) - c.cy) * c.iey : SID_INF;
        // z state of this lane's ray
        const int sz = v > 0.0f ? 1 : (v < 0.0f ? -1 : 0);
        const double ikz = sid_ikz(c, A, j), t0d = sid_t0(c);
        int cz = sid_zcell(tin, A, ikz, t0d);
        float tzn = sid_znext(cz, sz, A, ikz, t0d);
        float t = tin;
        for (;;) {
            const float tn = fminf(fminf(txn, tyn), tout);
            if (tn > t) {
                const float *col = vol_t + ((long)b * A.nx + a) * A.nz;
                float tt = t;
                while (tzn < tn) {
                    const float e = fmaxf(tzn, tt);
                    if ((unsigned)cz < (unsigned)A.nz) acc = fmaf(col[cz], e - tt, acc);
                    tt = e;
                    cz += sz;
                    tzn = sid_znext(cz, sz, A, ikz, t0d);
                }
                if ((unsigned)cz < (unsigned)A.nz) acc = fmaf(col[cz], tn - tt, acc);
                t = tn;
            }
            if (tn >= tout) break;
            if (txn <= tyn) {
                a += sx;
                if ((unsigned)a >= (unsigned)A.nx) break;
                txn = (sid_plane(a + (sx > 0), A.nx, A.hx) - c.cx) * c.iex;
            } else {
                b += sy;
                if ((unsigned)b >= (unsigned)A.ny) break;
                tyn = (sid_plane(b + (sy > 0), A.ny, A.hy) - c.cy) * c.iey;
            }
        }
    }
    if (j < A.nv) {
        const long view = vc / A.nu, i = vc - view * A.nu;
        out[(view * A.nv + j) * A.nu + i] = acc * sqrtf(fmaf(kz, kz, 1.0f));
    }
}

__global__ void __launch_bounds__(256) k_siddon_gather(const float *__restrict__ proj, const SidCol *__restrict__ cols,
                                                       const ViewParams *__restrict__ views, SidArgs A,
                                                       const float *__restrict__ fbase, float kappa,
                                                       float *__restrict__ out, float *__restrict__ out2) {
    const int ntx = (A.nx + 15) / 16, nzc = (A.nz + SID_TZ - 1) / SID_TZ;
    int w = cbct_xcd_remap(blockIdx.x, gridDim.x);
    const int zc = w % nzc;
    w /= nzc;
    const int a = (w % ntx) * 16 + (int)(threadIdx.x & 15), b = (w / ntx) * 16 + (int)(threadIdx.x >> 4);
    if (a >= A.nx || b >= A.ny) return;  // no barriers below
    const int c0 = zc * SID_TZ;
    float acc[SID_TZ];
    float zp[SID_TZ + 1];
#pragma unroll
    for (int k = 0; k < SID_TZ; k++) acc[k] = 0.0f;
#pragma unroll
    for (int k = 0; k <= SID_TZ; k++) zp[k] = sid_plane(c0 + k, A.nz, A.hz);
    const float xa = sid_plane(a, A.nx, A.hx), xb = sid_plane(a + 1, A.nx, A.hx);
    const float ya = sid_plane(b, A.ny, A.hy), yb = sid_plane(b + 1, A.ny, A.hy);
    const int zcell0 = sid_cell(0.0f, A.nz, A.hz);  // the cell of rays with v = 0
    const float iu = 0.5f * (float)(A.nu - 1), iv = 0.5f * (float)(A.nv - 1);
    const long vstride = (long)A.nv * A.nu;
    for (int view = 0; view < A.nviews; view++) {
        const ViewParams vp = views[view];
        // detector columns whose plane can cross the square: the fan projection of its corners
        float umin = SID_INF, umax = -SID_INF;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float x = (q & 1) ? xb : xa, y = (q & 2) ? yb : ya;
            const float u = A.sdd * (x * vp.sn - y * vp.cs) / (x * vp.cs + y * vp.sn + A.sad);
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
        }
        const int i0 = max((int)floorf(umin / A.pu + iu), 0), i1 = min((int)ceilf(umax / A.pu + iu), A.nu - 1);
        const float *pview = proj + (long)view * vstride;
        for (int i = i0; i <= i1; i++) {
            const SidCol c = cols[(long)view * A.nu + i];
            float ta = -c.t0, tb = c.lxy - c.t0;
            sid_slab(c.cx, c.iex, a, a + 1, A.nx, A.hx, ta, tb);
            sid_slab(c.cy, c.iey, b, b + 1, A.ny, A.hy, ta, tb);
            if (!(ta < tb)) continue;
            // rows meeting cell k: v in [zlo, zhi) / s for some s = (tau + t0) / lxy in [sa, sb]
            const float isa = 1.0f / ((ta + c.t0) * c.ilxy), isb = 1.0f / ((tb + c.t0) * c.ilxy);
            const float *pcol = pview + i;
#pragma unroll
            for (int k = 0; k < SID_TZ; k++) {
                if (c0 + k < A.nz) {
                    const float zlo = zp[k], zhi = zp[k + 1];
                    const float vmin = fminf(zlo * isa, zlo * isb), vmax = fmaxf(zhi * isa, zhi * isb);
                    const int j0 = max((int)floorf(vmin / A.pv + iv), 0);
                    const int j1 = min((int)ceilf(vmax / A.pv + iv), A.nv - 1);
                    float s = 0.0f;
                    for (int j = j0; j <= j1; j++) {
                        const float v = sid_row_v(j, A);
                        float lo, hi;
                        if (v != 0.0f) {
                            const double ikz = sid_ikz(c, A, j), t0d = sid_t0(c);
                            const float t1 = sid_zcross(c0 + k, A, ikz, t0d), t2 = sid_zcross(c0 + k + 1, A, ikz, t0d);
                            lo = fminf(t1, t2);
                            hi = fmaxf(t1, t2);
                        } else {
                            lo = c0 + k == zcell0 ? -SID_INF : SID_INF;
                            hi = SID_INF;
                        }
                        const float ov = fminf(tb, hi) - fmaxf(ta, lo);
                        if (ov > 0.0f) {
                            const float kz = v * c.ilxy;
                            s = fmaf(ov * sqrtf(fmaf(kz, kz, 1.0f)), pcol[(long)j * A.nu], s);
                        }
                    }
                    acc[k] += s;
                }
            }
        }
    }
    const long plane = (long)A.nx * A.ny;
#pragma unroll
    for (int k = 0; k < SID_TZ; k++)
        if (c0 + k < A.nz) {
            const long o = (c0 + k) * plane + (long)b * A.nx + a;
            const float v = fbase ? fmaf(-kappa, acc[k], fbase[o]) : acc[k];
            out[o] = v;
            if (out2) out2[o] = v;
        }
}

// Siddon forward by runs.  The xy line of a detector column is cut by the x and y grid planes
// into pieces, each inside one voxel column; all rows of the column share them.  Per chunk of KP
// pieces the work-group tabulates, for every z cell, Q_c at each piece start (the integral along
// the line of the cell's voxel values from the chunk start) and the piece's value, so that a ray's
// integral over a run [t0, t1) inside z cell c is Q_c(t1) - Q_c(t0), Q_c(t) = Q_c(piece start) +
// value (t - piece start).  A ray then costs O(z cells crossed + chunks) instead of O(pieces).
// The piece list is a stable merge of the x and y crossings, each crossing placed by its exact
// rank among the other axis's crossings; rows j and nv-1-j are mirror images (cell nz-1-c, the
// same crossings) and are summed by one thread.

// pieces per chunk for nz cells and a line of up to kmax pieces (0: the tables do not fit)
inline size_t sid_runs_lds(int kp, int nz, int kmax, int nwaves) {
    return (size_t)nz * (kp + 1) * 8 + (size_t)(2 * kmax + 2) * 4 + (size_t)(kmax + kp) * 8 + (size_t)nwaves * nz * 4;
}

// one float of the volume through a raw buffer resource at a byte offset; offsets past the end read 0
__device__ __forceinline__ float sid_ldv(__amdgpu_buffer_rsrc_t r, int voff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
}

struct SidLine {  // the crossings of one column's xy line, both axes
    float cx, cy, iex, iey;
    int nx, ny, a0, b0, sx, sy;
    float hx, hy;
    __device__ float tx(int m) const { return (sid_plane(a0 + (sx > 0) + sx * m, nx, hx) - cx) * iex; }
    __device__ float ty(int m) const { return (sid_plane(b0 + (sy > 0) + sy * m, ny, hy) - cy) * iey; }
    __device__ int mx_max() const { return iex == 0.0f ? 0 : (sx > 0 ? nx - a0 : a0 + 1); }
    __device__ int my_max() const { return iey == 0.0f ? 0 : (sy > 0 ? ny - b0 : b0 + 1); }
    // number of x crossings before t (strict: tx < t, else tx <= t); the estimate from the
    // crossing coordinate is corrected against the crossings themselves, which increase with m
    __device__ int count_x(float t, float ex, bool strict) const {
        const int mm = mx_max();
        if (mm == 0) return 0;
        const float pc = (cx + t * ex) / hx + 0.5f * (float)nx;
        int m = sx > 0 ? (int)floorf(pc) - a0 : a0 + 1 - (int)ceilf(pc);
        m = min(max(m, 0), mm);
        while (m > 0 && (strict ? tx(m - 1) >= t : tx(m - 1) > t)) m--;
        while (m < mm && (strict ? tx(m) < t : tx(m) <= t)) m++;
        return m;
    }
    __device__ int count_y(float t, float ey, bool strict) const {
        const int mm = my_max();
        if (mm == 0) return 0;
        const float pc = (cy + t * ey) / hy + 0.5f * (float)ny;
        int m = sy > 0 ? (int)floorf(pc) - b0 : b0 + 1 - (int)ceilf(pc);
        m = min(max(m, 0), mm);
        while (m > 0 && (strict ? ty(m - 1) >= t : ty(m - 1) > t)) m--;
        while (m < mm && (strict ? ty(m) < t : ty(m) <= t)) m++;
        return m;
    }
};

// The pieces of the line of column c inside the grid (entry tin < exit tout): pst[0 .. K] the
// piece starts (pst[K] = tout) and, when pof is given, pof[0 .. K-1] the element offset of each
// piece's voxel column (-1 outside the grid).  Piece 0 is the entry cell ln.a0, ln.b0; one piece
// follows every crossing, placed at its rank in the stable merge of the two axes' crossings (x
// first on ties), so piece k lies in voxel column (a0 + sx dx, b0 + sy dy) with dx + dy = k.  All
// threads of the work-group take part; the caller synchronises before reading.
__device__ int sid_piece_list(const SidCol &c, const SidArgs &A, float tin, float tout, int kmax, float *pst,
                              int *pof, int tid, int nthr, SidLine &ln) {
    ln.cx = c.cx; ln.cy = c.cy; ln.iex = c.iex; ln.iey = c.iey;
    ln.nx = A.nx; ln.ny = A.ny; ln.hx = A.hx; ln.hy = A.hy;
    ln.a0 = min(max(sid_cell(fmaf(tin, c.ex, c.cx), A.nx, A.hx), 0), A.nx - 1);
    ln.b0 = min(max(sid_cell(fmaf(tin, c.ey, c.cy), A.ny, A.hy), 0), A.ny - 1);
    if (c.iex == 0.0f) ln.a0 = sid_cell(c.cx, A.nx, A.hx);
    if (c.iey == 0.0f) ln.b0 = sid_cell(c.cy, A.ny, A.hy);
    ln.sx = c.ex > 0.0f ? 1 : -1;
    ln.sy = c.ey > 0.0f ? 1 : -1;
    const int mxc = ln.count_x(tout, c.ex, true), myc = ln.count_y(tout, c.ey, true);
    const int K = min(mxc + myc + 1, kmax);
    auto put = [&](int p, float t, int a, int b) {
        pst[p] = fminf(fmaxf(t, tin), tout);
        if (pof) pof[p] = (a >= 0 && a < A.nx && b >= 0 && b < A.ny) ? (b * A.nx + a) * A.nz : -1;
    };
    if (tid == 0) {
        put(0, tin, ln.a0, ln.b0);
        pst[K] = tout;
    }
    for (int m = tid; m < mxc; m += nthr) {
        const float t = ln.tx(m);
        const int p = m + ln.count_y(t, c.ey, true);  // y crossings strictly before: x first on ties
        if (p + 1 < K) put(p + 1, t, ln.a0 + ln.sx * (m + 1), ln.b0 + ln.sy * (p - m));
    }
    for (int n = tid; n < myc; n += nthr) {
        const float t = ln.ty(n);
        const int p = n + ln.count_x(t, c.ex, false);
        if (p + 1 < K) put(p + 1, t, ln.a0 + ln.sx * (p - n), ln.b0 + ln.sy * (n + 1));
    }
    return K;
}

template <int KP, int NPT>
__global__ void __launch_bounds__(256) k_siddon_forward_runs(const float *__restrict__ vol_t,
                                                             const SidCol *__restrict__ cols, SidArgs A, int kmax,
                                                             const float *__restrict__ ysub, float *__restrict__ out,
                                                             double *__restrict__ partials) {
    extern __shared__ float4 lds4[];
    constexpr int S = KP + 1;  // per cell: (Q at piece start, piece value) for KP pieces, then (chunk total, 0)
    const int nz = A.nz;
    float2 *tab = reinterpret_cast<float2 *>(lds4);
    float *pst = reinterpret_cast<float *>(tab + nz * S);  // piece starts, pst[K] = exit
    int *pof = reinterpret_cast<int *>(pst + kmax + 1);    // voxel-column element offset, -1 outside
    float2 *pk = reinterpret_cast<float2 *>(pof + kmax + 1);  // [kmax + KP]: (length, byte offset bits)
    float *tot = reinterpret_cast<float *>(pk + kmax + KP);  // [wave][nz]: slice totals

    const int vc = cbct_xcd_remap(blockIdx.x, gridDim.x);  // view * nu + column
    const int view = vc / A.nu, i = vc - view * A.nu;
    const SidCol c = cols[vc];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    const int npairs = (A.nv + 1) >> 1;

    float tin = -c.t0, tout = c.lxy - c.t0;
    sid_slab(c.cx, c.iex, 0, A.nx, A.nx, A.hx, tin, tout);
    sid_slab(c.cy, c.iey, 0, A.ny, A.ny, A.hy, tin, tout);
    float acc[NPT], accm[NPT];
#pragma unroll
    for (int p = 0; p < NPT; p++) acc[p] = accm[p] = 0.0f;

    if (tin < tout) {  // uniform over the work-group
        SidLine ln;
        const int K = sid_piece_list(c, A, tin, tout, kmax, pst, pof, tid, nthr, ln);
        __syncthreads();
        // per piece: length and the byte offset of its voxel column; outside the grid, and past the
        // last piece up to the chunk edge, the volume's size: plus a cell's offset that stays past
        // the end (reads 0) and below 2^31 (the launcher checks the size)
        const int kr = (K + KP - 1) / KP * KP;
        const int vbytes = A.nx * A.ny * nz * 4;
        for (int k = tid; k < kr; k += nthr) {
            const bool in = k < K && pof[k] >= 0;
            pk[k] = make_float2(k < K ? pst[k + 1] - pst[k] : 0.0f, __int_as_float(in ? pof[k] * 4 : vbytes));
        }
        const __amdgpu_buffer_rsrc_t vrs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(vol_t), 0, A.nx * A.ny * nz * 4, 0x00020000);
        const float ihx = 1.0f / A.hx, ihy = 1.0f / A.hy;

        // rays: pair p = row j (v <= 0) and its mirror nv - 1 - j; z state of row j
        double ikz[NPT];
        const double t0d = sid_t0(c);
        int cz[NPT], szr[NPT];
        float tzn[NPT];
#pragma unroll
        for (int p = 0; p < NPT; p++) {
            const int j = min(tid + p * nthr, npairs - 1);
            const float v = sid_row_v(j, A);
            szr[p] = v > 0.0f ? 1 : (v < 0.0f ? -1 : 0);
            ikz[p] = sid_ikz(c, A, j);
            cz[p] = sid_zcell(tin, A, ikz[p], t0d);
            tzn[p] = sid_znext(cz[p], szr[p], A, ikz[p], t0d);
        }
        const int sc = ((KP + nw - 1) / nw + 7) & ~7;
        const int ka = min(wave * sc, KP), kb = min(ka + sc, KP);
        for (int k0 = 0; k0 < K; k0 += KP) {
            const int kn = min(KP, K - k0);
            __syncthreads();  // the piece list is complete / the previous chunk's rays are done
            // Q of this wave's slice of pieces (whole groups of 8; pieces past the list have length
            // 0 and read 0), lane = z cell; a group's loads are in flight together
            constexpr int GB = 8;
            for (int cc = lane; cc < nz; cc += 64) {
                float q = 0.0f;
                float2 *row = tab + cc * S;
                const int c4 = cc * 4;
                for (int k = ka; k < kb; k += GB) {
                    float2 pe[GB];
                    float f[GB];
#pragma unroll
                    for (int u = 0; u < GB; u++) {
                        pe[u] = pk[k0 + k + u];
                        f[u] = sid_ldv(vrs, __float_as_int(pe[u].y) + c4);
                    }
#pragma unroll
                    for (int u = 0; u < GB; u++) {
                        row[k + u] = make_float2(q, f[u]);
                        q = fmaf(f[u], pe[u].x, q);
                    }
                }
                tot[wave * nz + cc] = q;
            }
            __syncthreads();
            for (int cc = lane; cc < nz; cc += 64) {
                float off = 0.0f;
                for (int w2 = 0; w2 < wave; w2++) off += tot[w2 * nz + cc];
                if (wave > 0)
                    for (int k = ka; k < kb; k++) tab[cc * S + k].x += off;
                if (wave == nw - 1) {  // the chunk's total for every cell
                    float all = off;
                    for (int w2 = wave; w2 < nw; w2++) all += tot[w2 * nz + cc];
                    tab[cc * S + KP] = make_float2(all, 0.0f);
                }
            }
            __syncthreads();
            const float T1 = pst[k0 + kn];  // chunk end
#pragma unroll
            for (int p = 0; p < NPT; p++) {
                int z = cz[p];
                float tz = tzn[p];
                float qa = 0.0f, qam = 0.0f;  // Q of the current cells at the run start (chunk start: 0)
                float r = 0.0f, rm = 0.0f;
                for (;;) {
                    const bool cross = tz < T1;
                    const int zm = nz - 1 - z;
                    const int zc = min(max(z, 0), nz - 1), zmc = min(max(zm, 0), nz - 1);
                    float q1, q1m;
                    int k = KP;
                    float dt = 0.0f;
                    if (cross) {
                        // the piece holding tz: one piece per x or y step from the entry
                        // (a multiply for the cell: off by one only within rounding of a plane, where
                        // the neighbouring piece's Q agrees)
                        const int a = c.iex != 0.0f
                                          ? min(max((int)floorf(fmaf(fmaf(tz, c.ex, c.cx), ihx, 0.5f * A.nx)), 0), A.nx - 1)
                                          : ln.a0;
                        const int b = c.iey != 0.0f
                                          ? min(max((int)floorf(fmaf(fmaf(tz, c.ey, c.cy), ihy, 0.5f * A.ny)), 0), A.ny - 1)
                                          : ln.b0;
                        k = min(max(abs(a - ln.a0) + abs(b - ln.b0) - k0, 0), kn - 1);
                        dt = tz - pst[k0 + k];
                    }
                    const float2 e1 = tab[zc * S + k], e1m = tab[zmc * S + k];
                    q1 = fmaf(e1.y, dt, e1.x);
                    q1m = fmaf(e1m.y, dt, e1m.x);
                    if (z == zc) r += q1 - qa;
                    if (zm == zmc) rm += q1m - qam;
                    if (!cross) break;
                    // into the next z cell at tz
                    z += szr[p];
                    const int zn = nz - 1 - z;
                    const int znc = min(max(z, 0), nz - 1), znmc = min(max(zn, 0), nz - 1);
                    const float2 e2 = tab[znc * S + k], e2m = tab[znmc * S + k];
                    qa = fmaf(e2.y, dt, e2.x);
                    qam = fmaf(e2m.y, dt, e2m.x);
                    tz = sid_znext(z, szr[p], A, ikz[p], t0d);
                }
                cz[p] = z;
                tzn[p] = tz;
                acc[p] += r;
                accm[p] += rm;
            }
        }
    }
    double part = 0.0;
#pragma unroll
    for (int p = 0; p < NPT; p++) {
        const int j = tid + p * nthr;
        if (j < npairs) {
            const int jm = A.nv - 1 - j;
            const float kz = sid_row_v(j, A) * c.ilxy;
            const float w = sqrtf(fmaf(kz, kz, 1.0f));  // the mirror's weight is the same
            const long o1 = ((long)view * A.nv + j) * A.nu + i, o2 = ((long)view * A.nv + jm) * A.nu + i;
            float r1 = acc[p] * w, r2 = accm[p] * w;
            if (ysub) {  // residual and its sum of squares
                r1 -= ysub[o1];
                r2 -= ysub[o2];
                part += (double)r1 * (double)r1;
                if (jm != j) part += (double)r2 * (double)r2;
            }
            out[o1] = r1;
            if (jm != j) out[o2] = r2;
        }
    }
    if (partials) {
        __shared__ double wsum[4];
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
        if (lane == 0) wsum[wave] = part;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int w2 = 0; w2 < nw; w2++) sum += wsum[w2];
            partials[vc] = sum;
        }
    }
}

// Siddon transpose, pass 1: for every piece k of column i's line and z cell c,
//   Z_k(c) = sum_j w_j y_j |piece k  n  {tau : ray j in cell c}|,
// as Z_k(c) = W_{c+1}(k) - W_c(k), W_p(k) the integral over piece k of U_p(tau), the sum of w y over
// the rows whose ray lies below z plane p at tau.  Those rows are a prefix j < J_p(tau) of the rows
// (sorted by detector height v: ray j is below the plane where v_j < z_p lxy / (tau + t0)), and J
// changes inside a piece only for the few rows whose ray crosses the plane there:
//   W_p = len A(J_lo) + sum over J_lo <= j < J_hi of w_j y_j (time of ray j below the plane),
// A the prefix sum of w y over the rows (accumulated in FP64), the crossing time from the same
// expression as the forward kernel's.  Z is formed as len (A(J_lo, p+1) - A(J_lo, p)) + (difference
// of the crossing terms), so FP32 suffices.  One work-group per (view, column); lane = piece, 16
// cells at a time staged in LDS and stored as whole 64-byte runs; profiles go to
// Z[(view nu + i) kmax + k][c], and rec[view nu + i] = (entry cell a0, b0, piece count K).
constexpr int SPC = 16;  // cells per staged block of the profiles

__global__ void __launch_bounds__(256) k_sid_profiles(const float *__restrict__ proj, const SidCol *__restrict__ cols,
                                                      SidArgs A, int kmax, float *__restrict__ Z,
                                                      int4 *__restrict__ rec) {
    extern __shared__ float ldsf[];
    const int nv = A.nv, nz = A.nz;
    float *Af = ldsf;                // [nv + 1]: prefix of w y
    float *wyf = Af + nv + 1;        // [nv]: w y
    double *ivd = reinterpret_cast<double *>(wyf + nv + 1);  // [nv] (8-byte aligned): lxy / v, 0 for v = 0
    float *pst = reinterpret_cast<float *>(ivd + nv);  // [kmax + 1]
    float *stg = pst + kmax + 1;     // [4][64][SPC + 1]
    const int vc = cbct_xcd_remap(blockIdx.x, gridDim.x);
    const int view = vc / A.nu, i = vc - view * A.nu;
    const SidCol c = cols[vc];
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
    float tin = -c.t0, tout = c.lxy - c.t0;
    sid_slab(c.cx, c.iex, 0, A.nx, A.nx, A.hx, tin, tout);
    sid_slab(c.cy, c.iey, 0, A.ny, A.ny, A.hy, tin, tout);
    if (!(tin < tout)) {  // uniform: the line misses the grid
        if (tid == 0) rec[vc] = make_int4(0, 0, 0, 0);
        return;
    }
    for (int j = tid; j < nv; j += nthr) {
        const float v = sid_row_v(j, A), kz = v * c.ilxy;
        wyf[j] = sqrtf(fmaf(kz, kz, 1.0f)) * proj[((long)view * nv + j) * A.nu + i];
        ivd[j] = sid_ikz(c, A, j);
    }
    __syncthreads();
    if (tid < 64) {  // prefix over the rows in FP64, lane l taking rows [l R, (l + 1) R)
        const int R = (nv + 63) / 64;
        double s = 0.0;
        for (int r = 0; r < R; r++) {
            const int j = lane * R + r;
            if (j < nv) s += (double)wyf[j];
        }
        double incl = s;
        for (int o = 1; o < 64; o <<= 1) {
            const double t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        double run = incl - s;
        for (int r = 0; r < R; r++) {
            const int j = lane * R + r;
            if (j < nv) {
                Af[j] = (float)run;
                run += (double)wyf[j];
            }
        }
        if (lane == 63) Af[nv] = (float)incl;
    }
    SidLine ln;
    const int K = sid_piece_list(c, A, tin, tout, kmax, pst, nullptr, tid, nthr, ln);
    if (tid == 0) rec[vc] = make_int4(ln.a0, ln.b0, K, 0);
    __syncthreads();
    const double t0d = sid_t0(c);
    float *Zl = Z + (long)vc * kmax * nz;
    float *st = stg + wave * 64 * (SPC + 1);
    const float cj = 0.5f * (float)(nv - 1), ipv = 1.0f / A.pv;
    const bool vec = (nz & 3) == 0;
    for (int kb = wave * 64; kb < K; kb += nw * 64) {  // uniform per wave
        const int k = kb + lane;
        const bool live = k < K;
        const float ta = live ? pst[k] : 0.0f, tb = live ? pst[k + 1] : 0.0f, len = tb - ta;
        const float isa = 1.0f / ((ta + c.t0) * c.ilxy), isb = 1.0f / ((tb + c.t0) * c.ilxy);
        // (A(J_lo), crossing term) at plane p
        auto plane_terms = [&](int p, float &alo, float &part) {
            const float zp = sid_plane(p, nz, A.hz);
            const float xa = zp * isa, xb = zp * isb;
            // rows with v_j < x: j < x / pv + (nv - 1) / 2
            const int jl = (int)fminf(fmaxf(ceilf(fmaf(fminf(xa, xb), ipv, cj)), 0.0f), (float)nv);
            const int jh = (int)fminf(fmaxf(ceilf(fmaf(fmaxf(xa, xb), ipv, cj)), 0.0f), (float)nv);
            alo = Af[jl];
            part = 0.0f;
            for (int j = jl; j < jh; j++) {
                const float th = sid_zcross(p, A, ivd[j], t0d);  // the forward kernel's crossing of plane p
                part = fmaf(wyf[j], fminf(fmaxf(zp > 0.0f ? th - ta : tb - th, 0.0f), len), part);
            }
        };
        float pa, pp;
        plane_terms(0, pa, pp);
        for (int c0 = 0; c0 < nz; c0 += SPC) {
#pragma unroll 4
            for (int u = 0; u < SPC; u++) {
                if (c0 + u < nz) {
                    float na, np;
                    plane_terms(c0 + u + 1, na, np);
                    st[lane * (SPC + 1) + u] = fmaf(len, na - pa, np - pp);
                    pa = na;
                    pp = np;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // the wave's 64 pieces x SPC cells: lane pairs (piece, group of 4 cells)
            for (int r = lane; r < 64 * (SPC / 4); r += 64) {
                const int pc = r / (SPC / 4), g4 = (r - pc * (SPC / 4)) * 4;
                const int kk = kb + pc, cc = c0 + g4;
                if (kk < K && cc < nz) {
                    const float *sv = st + pc * (SPC + 1) + g4;
                    float *dst = Zl + (long)kk * nz + cc;
                    if (vec) {
                        // non-temporal: pass 2 reads each line once (P_s^T 2.29 against 2.41 ms at
                        // 512x512x64 / 40 views)
                        typedef float v4f __attribute__((ext_vector_type(4)));
                        const v4f t = {sv[0], sv[1], sv[2], sv[3]};
                        __builtin_nontemporal_store(t, reinterpret_cast<v4f *>(dst));
                    } else {
                        for (int u = 0; u < 4 && cc + u < nz; u++) dst[u] = sv[u];
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Siddon transpose, pass 2: a thread owns SGC z cells of one voxel column (a, b); per view and per
// detector column whose line crosses the column's square, the crossing is piece k = |a - a0| +
// |b - b0| of that line, whose profile it adds.  Work-group: 8 x 8 voxel columns x 4 groups of SGC
// cells (blockIdx.y picks the z block of 4 SGC cells).  Every voxel is written once; no atomics.
constexpr int SGC = 16;

__global__ void __launch_bounds__(256) k_sid_gather_pieces(const float *__restrict__ Z, const int4 *__restrict__ rec,
                                                           const SidCol *__restrict__ cols,
                                                           const ViewParams *__restrict__ views, SidArgs A, int kmax,
                                                           const float *__restrict__ fbase, float kappa,
                                                           float *__restrict__ out, float *__restrict__ out2) {
    const int ntx = (A.nx + 7) / 8;
    const int w = cbct_xcd_remap(blockIdx.x, gridDim.x);
    const int g = threadIdx.x & 3, q = threadIdx.x >> 2;
    const int a = (w % ntx) * 8 + (q & 7), b = (w / ntx) * 8 + (q >> 3);
    const int c0 = (blockIdx.y * 4 + g) * SGC;
    if (a >= A.nx || b >= A.ny || c0 >= A.nz) return;  // no barriers below
    const int nz = A.nz;
    const bool vec = (nz & 3) == 0;
    float acc[SGC];
#pragma unroll
    for (int u = 0; u < SGC; u++) acc[u] = 0.0f;
    const float xa = sid_plane(a, A.nx, A.hx), xb = sid_plane(a + 1, A.nx, A.hx);
    const float ya = sid_plane(b, A.ny, A.hy), yb = sid_plane(b + 1, A.ny, A.hy);
    const float iu = 0.5f * (float)(A.nu - 1);
    for (int view = 0; view < A.nviews; view++) {
        const ViewParams vp = views[view];
        float umin = SID_INF, umax = -SID_INF;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const float x = (r & 1) ? xb : xa, y = (r & 2) ? yb : ya;
            const float u = A.sdd * (x * vp.sn - y * vp.cs) / (x * vp.cs + y * vp.sn + A.sad);
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
        }
        const int i0 = max((int)floorf(umin / A.pu + iu), 0), i1 = min((int)ceilf(umax / A.pu + iu), A.nu - 1);
        for (int i = i0; i <= i1; i++) {
            const long vc = (long)view * A.nu + i;
            const SidCol c = cols[vc];
            float ta = -c.t0, tb = c.lxy - c.t0;
            sid_slab(c.cx, c.iex, a, a + 1, A.nx, A.hx, ta, tb);
            sid_slab(c.cy, c.iey, b, b + 1, A.ny, A.hy, ta, tb);
            if (!(ta < tb)) continue;
            const int4 r = rec[vc];
            const int k = abs(a - r.x) + abs(b - r.y);
            if (k >= r.z) continue;
            const float *zl = Z + (vc * kmax + k) * nz + c0;
            if (vec && c0 + SGC <= nz) {
#pragma unroll
                for (int u = 0; u < SGC; u += 4) {
                    const float4 z4 = *reinterpret_cast<const float4 *>(zl + u);
                    acc[u] += z4.x;
                    acc[u + 1] += z4.y;
                    acc[u + 2] += z4.z;
                    acc[u + 3] += z4.w;
                }
            } else {
#pragma unroll
                for (int u = 0; u < SGC; u++)
                    if (c0 + u < nz) acc[u] += zl[u];
            }
        }
    }
    const long plane = (long)A.nx * A.ny;
#pragma unroll
    for (int u = 0; u < SGC; u++)
        if (c0 + u < nz) {
            const long o = (c0 + u) * plane + (long)b * A.nx + a;
            const float v = fbase ? fmaf(-kappa, acc[u], fbase[o]) : acc[u];
            out[o] = v;
            if (out2) out2[o] = v;
        }
}

// residual of the per-ray forward: one work-group per detector column, out = out - ysub in
// place and partials[view * nu + i] = sum over the column's rows of its square
__global__ void __launch_bounds__(256) k_sid_residual(const float *__restrict__ ysub, float *__restrict__ out,
                                                      double *__restrict__ partials, int nu, int nv) {
    __shared__ double wsum[4];
    const long vc = blockIdx.x;
    const long view = vc / nu, i = vc - view * nu;
    double part = 0.0;
    for (int j = threadIdx.x; j < nv; j += blockDim.x) {
        const long o = (view * nv + j) * nu + i;
        const float r = out[o] - ysub[o];
        out[o] = r;
        part += (double)r * (double)r;
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0 && partials) partials[vc] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

SidArgs sid_args(const Level &L) {
    SidArgs A;
    A.nx = L.nx; A.ny = L.ny; A.nz = L.nz; A.nu = L.nu; A.nv = L.nv; A.nviews = L.nviews;
    A.hx = (float)L.hx; A.hy = (float)L.hy; A.hz = (float)L.hz; A.pu = (float)L.pu; A.pv = (float)L.pv;
    A.sad = (float)L.sad; A.sdd = (float)L.sdd;
    A.hzd = L.hz; A.pvd = L.pv;
    return A;
}

}  // namespace

template <int KP>
cbct_status launch_sid_runs(const Level &L, const float *vol_t, const float *ysub, float *out, double *partials,
                            hipStream_t s, int npt, int block, int kmax, size_t lds) {
    const dim3 grid((unsigned)((long)L.nviews * L.nu));
    if (npt == 1)
        hipLaunchKernelGGL((k_siddon_forward_runs<KP, 1>), grid, dim3(block), lds, s, vol_t, L.d_sid, sid_args(L), kmax, ysub, out, partials);
    else if (npt == 2)
        hipLaunchKernelGGL((k_siddon_forward_runs<KP, 2>), grid, dim3(block), lds, s, vol_t, L.d_sid, sid_args(L), kmax, ysub, out, partials);
    else if (npt == 4)
        hipLaunchKernelGGL((k_siddon_forward_runs<KP, 4>), grid, dim3(block), lds, s, vol_t, L.d_sid, sid_args(L), kmax, ysub, out, partials);
    else
        hipLaunchKernelGGL((k_siddon_forward_runs<KP, 8>), grid, dim3(block), lds, s, vol_t, L.d_sid, sid_args(L), kmax, ysub, out, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_siddon_forward_runs launch");
    return CBCT_OK;
}

cbct_status cbct_launch_forward_siddon(const Level &L, const float *vol_t, const float *ysub, float *out,
                                       double *partials, hipStream_t s) {
    {
        // the run-summing kernel when its tables fit: rays in mirrored pairs, up to 256 threads
        const int npairs = (L.nv + 1) / 2;
        int npt = 1;
        while ((npairs + npt - 1) / npt > 256) npt *= 2;
        const int block = (((npairs + npt - 1) / npt + 63) / 64) * 64;
        const int kmax = L.nx + L.ny + 3;
        constexpr size_t budget = 48 * 1024;
        const bool fits32 = ((long)L.nx * L.ny * L.nz + (long)L.nz) * 4 < (1L << 31);  // 32-bit byte offsets
        // With two or more waves, which split each chunk's table build into slices of whole groups
        // of 8 pieces, the largest chunk of equal slices (a multiple of 8 x waves, at most 64) whose
        // tables fit 32 KB (five work-groups per CU): at 512x512x64 / 40 views (three waves) 24
        // pieces took 1.06 ms per P_s against 1.10 with 40, 1.16 with 16 and 1.27 with 32 (slices
        // 16, 16 and none, four work-groups per CU).  Otherwise the largest of 64, 32 or 16 within
        // 48 KB.
        const int nw = block / 64, step = 8 * nw;
        if (fits32 && npt <= 8 && nw >= 2) {
            for (int kp = 64 / step * step; kp >= step; kp -= step) {
                const size_t l = sid_runs_lds(kp, L.nz, kmax, nw);
                if (l > 32 * 1024) continue;
                switch (kp) {
                    case 64: return launch_sid_runs<64>(L, vol_t, ysub, out, partials, s, npt, block, kmax, l);
                    case 48: return launch_sid_runs<48>(L, vol_t, ysub, out, partials, s, npt, block, kmax, l);
                    case 32: return launch_sid_runs<32>(L, vol_t, ysub, out, partials, s, npt, block, kmax, l);
                    case 24: return launch_sid_runs<24>(L, vol_t, ysub, out, partials, s, npt, block, kmax, l);
                    case 16: return launch_sid_runs<16>(L, vol_t, ysub, out, partials, s, npt, block, kmax, l);
                    default: break;
                }
            }
        }
        if (fits32 && npt <= 8 && sid_runs_lds(64, L.nz, kmax, block / 64) <= budget)
            return launch_sid_runs<64>(L, vol_t, ysub, out, partials, s, npt, block, kmax,
                                         sid_runs_lds(64, L.nz, kmax, block / 64));
        if (fits32 && npt <= 8 && sid_runs_lds(32, L.nz, kmax, block / 64) <= budget)
            return launch_sid_runs<32>(L, vol_t, ysub, out, partials, s, npt, block, kmax,
                                         sid_runs_lds(32, L.nz, kmax, block / 64));
        if (fits32 && npt <= 8 && sid_runs_lds(16, L.nz, kmax, block / 64) <= budget)
            return launch_sid_runs<16>(L, vol_t, ysub, out, partials, s, npt, block, kmax,
                                         sid_runs_lds(16, L.nz, kmax, block / 64));
    }
    const int nchunk = (L.nv + 63) / 64;
    const long items = (long)L.nviews * L.nu * nchunk;
    const long blocks = (items + 3) / 4;
    if (blocks > 0x7fffffffL) return cbct_set_error(CBCT_ERR_INVALID_ARG, "forward_siddon: grid too large");
    hipLaunchKernelGGL(k_siddon_forward, dim3((unsigned)blocks), dim3(256), 0, s, vol_t, L.d_sid, sid_args(L), nchunk,
                       out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_siddon_forward launch");
    if (ysub) {
        hipLaunchKernelGGL(k_sid_residual, dim3((unsigned)((long)L.nviews * L.nu)), dim3(256), 0, s, ysub, out, partials,
                           L.nu, L.nv);
        e = hipGetLastError();
        if (e != hipSuccess) return cbct_hip_error(e, "k_sid_residual launch");
    }
    return CBCT_OK;
}

size_t cbct_adjoint_siddon_ws_bytes(const Level &L) {
    const size_t lines = (size_t)L.nviews * L.nu;
    const size_t kmax = (size_t)L.nx + L.ny + 3;
    return ((lines * kmax * L.nz * 4 + 255) & ~(size_t)255) + lines * 16;
}

cbct_status cbct_launch_adjoint_siddon(const Level &L, const float *proj, const float *fbase, float kappa, float *out,
                                       void *ws, hipStream_t s, float *out2) {
    const int kmax = L.nx + L.ny + 3;
    // Af, wyf (2 nv + 1 floats, padded to a whole double), ivd (nv doubles), pst, the staging blocks
    const size_t lds = (size_t)(2 * L.nv + 2) * 4 + (size_t)L.nv * 8 + (size_t)(kmax + 1) * 4 +
                       (size_t)4 * 64 * (16 + 1) * 4;
    if (lds <= 64 * 1024) {
        const size_t lines = (size_t)L.nviews * L.nu;
        float *Z = static_cast<float *>(ws);
        int4 *rec = reinterpret_cast<int4 *>(static_cast<char *>(ws) + ((lines * kmax * L.nz * 4 + 255) & ~(size_t)255));
        hipLaunchKernelGGL(k_sid_profiles, dim3((unsigned)lines), dim3(256), lds, s, proj, L.d_sid, sid_args(L), kmax, Z,
                           rec);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return cbct_hip_error(e, "k_sid_profiles launch");
        const dim3 grid((unsigned)(((L.nx + 7) / 8) * ((L.ny + 7) / 8)), (unsigned)((L.nz + 4 * SGC - 1) / (4 * SGC)));
        hipLaunchKernelGGL(k_sid_gather_pieces, grid, dim3(256), 0, s, Z, rec, L.d_sid, L.d_views, sid_args(L), kmax,
                           fbase, kappa, out, out2);
        e = hipGetLastError();
        if (e != hipSuccess) return cbct_hip_error(e, "k_sid_gather_pieces launch");
        return CBCT_OK;
    }
    const long blocks = (long)((L.nx + 15) / 16) * ((L.ny + 15) / 16) * ((L.nz + SID_TZ - 1) / SID_TZ);
    if (blocks > 0x7fffffffL) return cbct_set_error(CBCT_ERR_INVALID_ARG, "adjoint_siddon: grid too large");
    hipLaunchKernelGGL(k_siddon_gather, dim3((unsigned)blocks), dim3(256), 0, s, proj, L.d_sid, L.d_views, sid_args(L),
                       fbase, kappa, out, out2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_siddon_gather launch");
    return CBCT_OK;
}
