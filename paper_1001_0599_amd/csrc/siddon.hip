// Siddon's exact radiological path (the ray tracer of Section II.C.2, also the paper's data
// simulator in Section III.A) as a projector pair: every voxel is constant on its cube and a ray's
// value is the sum over voxels of (length of the ray inside the cube) x (voxel value).
//
// Parameterisation.  All rays of one detector column lie in one vertical plane and share its
// transverse (xy) line.  tau is the transverse distance along that line from C, the line's closest
// approach to the rotation axis (|tau| stays within the grid's half diagonal, so FP32 crossing
// parameters are accurate to ~1e-5 mm); the source sits at tau = -t0, the detector at lxy - t0.
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

// tau at which a ray with dz/dtau = v / lxy (ikz = lxy / v) crosses z plane p
__device__ __forceinline__ float sid_zcross(int p, const SidArgs &A, float ikz, float t0) {
    return sid_plane(p, A.nz, A.hz) * ikz - t0;
}

// tau of the next z crossing of a lane in cell cz moving by sz (+-1, 0): none once it has left the grid
__device__ __forceinline__ float sid_znext(int cz, int sz, const SidArgs &A, float ikz, float t0) {
    if (sz > 0) return cz < A.nz ? sid_zcross(cz + 1, A, ikz, t0) : SID_INF;
    if (sz < 0) return cz >= 0 ? sid_zcross(cz, A, ikz, t0) : SID_INF;
    return SID_INF;
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
        const float ikz = v != 0.0f ? c.lxy * (1.0f / v) : 0.0f;
        int cz = min(max(sid_cell((tin + c.t0) * kz, A.nz, A.hz), -1), A.nz);
        float tzn = sid_znext(cz, sz, A, ikz, c.t0);
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
                    tzn = sid_znext(cz, sz, A, ikz, c.t0);
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
                                                       float *__restrict__ out) {
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
                            const float ikz = c.lxy * (1.0f / v);
                            const float t1 = sid_zcross(c0 + k, A, ikz, c.t0), t2 = sid_zcross(c0 + k + 1, A, ikz, c.t0);
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
        if (c0 + k < A.nz) out[(c0 + k) * plane + (long)b * A.nx + a] = acc[k];
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
    return (size_t)nz * (kp + 1) * 8 + (size_t)(2 * kmax + 2) * 4 + (size_t)nwaves * nz * 4;
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

template <int KP, int NPT>
__global__ void __launch_bounds__(256) k_siddon_forward_runs(const float *__restrict__ vol_t,
                                                             const SidCol *__restrict__ cols, SidArgs A, int kmax,
                                                             float *__restrict__ out) {
    extern __shared__ float4 lds4[];
    constexpr int S = KP + 1;  // per cell: (Q at piece start, piece value) for KP pieces, then (chunk total, 0)
    const int nz = A.nz;
    float2 *tab = reinterpret_cast<float2 *>(lds4);
    float *pst = reinterpret_cast<float *>(tab + nz * S);  // piece starts, pst[K] = exit
    int *pof = reinterpret_cast<int *>(pst + kmax + 1);    // voxel-column element offset, -1 outside
    float *tot = reinterpret_cast<float *>(pof + kmax + 1);  // [wave][nz]: slice totals

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
        // the piece list: piece 0 at the entry, then one piece after every crossing
        auto put = [&](int p, float t, int a, int b) {
            pst[p] = fminf(fmaxf(t, tin), tout);
            const bool in = a >= 0 && a < A.nx && b >= 0 && b < A.ny;
            pof[p] = in ? (b * A.nx + a) * nz : -1;
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

        // rays: pair p = row j (v <= 0) and its mirror nv - 1 - j; z state of row j
        float ikz[NPT], t0r[NPT];
        int cz[NPT], szr[NPT];
        float tzn[NPT];
#pragma unroll
        for (int p = 0; p < NPT; p++) {
            const int j = tid + p * nthr;
            const float v = sid_row_v(min(j, npairs - 1), A);
            szr[p] = v > 0.0f ? 1 : (v < 0.0f ? -1 : 0);
            ikz[p] = v != 0.0f ? c.lxy * (1.0f / v) : 0.0f;
            t0r[p] = tin;
            cz[p] = min(max(sid_cell((tin + c.t0) * (v * c.ilxy), A.nz, A.hz), -1), A.nz);
            tzn[p] = sid_znext(cz[p], szr[p], A, ikz[p], c.t0);
        }
        const int sc = ((KP + nw - 1) / nw + 7) & ~7;
        const int ka = min(wave * sc, KP), kb = min(ka + sc, KP);
        const int olast = (A.nx * A.ny - 1) * nz;  // last voxel column's offset
        for (int k0 = 0; k0 < K; k0 += KP) {
            const int kn = min(KP, K - k0);
            __syncthreads();  // the piece list is complete / the previous chunk's rays are done
            // Q of this wave's slice of pieces, lane = z cell; groups of 8 pieces keep their loads
            // in flight together
            const int kbe = min(kb, kn);
            for (int cc = lane; cc < nz; cc += 64) {
                float q = 0.0f;
                float2 *row = tab + cc * S;
                for (int k = ka; k < kbe; k += 8) {
                    float f[8];
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        const int o = (k + u < kbe) ? pof[k0 + k + u] : -1;
                        f[u] = (o >= 0 && o <= olast) ? vol_t[o + cc] : 0.0f;
                    }
#pragma unroll
                    for (int u = 0; u < 8; u++) {
                        if (k + u < kbe) {
                            const float len = pst[k0 + k + u + 1] - pst[k0 + k + u];
                            row[k + u] = make_float2(q, f[u]);
                            q = fmaf(f[u], len, q);
                        }
                    }
                }
                tot[wave * nz + cc] = q;
            }
            __syncthreads();
            for (int cc = lane; cc < nz; cc += 64) {
                float off = 0.0f;
                for (int w2 = 0; w2 < wave; w2++) off += tot[w2 * nz + cc];
                if (wave > 0)
                    for (int k = ka; k < kbe; k++) tab[cc * S + k].x += off;
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
                        const int a = c.iex != 0.0f ? min(max(sid_cell(fmaf(tz, c.ex, c.cx), A.nx, A.hx), 0), A.nx - 1)
                                                    : ln.a0;
                        const int b = c.iey != 0.0f ? min(max(sid_cell(fmaf(tz, c.ey, c.cy), A.ny, A.hy), 0), A.ny - 1)
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
                    tz = sid_znext(z, szr[p], A, ikz[p], c.t0);
                }
                cz[p] = z;
                tzn[p] = tz;
                acc[p] += r;
                accm[p] += rm;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < NPT; p++) {
        const int j = tid + p * nthr;
        if (j < npairs) {
            const int jm = A.nv - 1 - j;
            const float kz = sid_row_v(j, A) * c.ilxy;
            const float w = sqrtf(fmaf(kz, kz, 1.0f));  // the mirror's weight is the same
            out[((long)view * A.nv + j) * A.nu + i] = acc[p] * w;
            if (jm != j) out[((long)view * A.nv + jm) * A.nu + i] = accm[p] * w;
        }
    }
}

SidArgs sid_args(const Level &L) {
    SidArgs A;
    A.nx = L.nx; A.ny = L.ny; A.nz = L.nz; A.nu = L.nu; A.nv = L.nv; A.nviews = L.nviews;
    A.hx = (float)L.hx; A.hy = (float)L.hy; A.hz = (float)L.hz; A.pu = (float)L.pu; A.pv = (float)L.pv;
    A.sad = (float)L.sad; A.sdd = (float)L.sdd;
    return A;
}

}  // namespace

template <int KP>
cbct_status launch_sid_runs(const Level &L, const float *vol_t, float *out, hipStream_t s, int npt, int block,
                            int kmax, size_t lds) {
    const dim3 grid((unsigned)((long)L.nviews * L.nu));
    if (npt == 1)
        hipLaunchKernelGGL((k_siddon_forward_runs<KP, 1>), grid, dim3(block), lds, s, vol_t, L.d_sid, sid_args(L), kmax, out);
    else if (npt == 2)
        hipLaunchKernelGGL((k_siddon_forward_runs<KP, 2>), grid, dim3(block), lds, s, vol_t, L.d_sid, sid_args(L), kmax, out);
    else if (npt == 4)
        hipLaunchKernelGGL((k_siddon_forward_runs<KP, 4>), grid, dim3(block), lds, s, vol_t, L.d_sid, sid_args(L), kmax, out);
    else
        hipLaunchKernelGGL((k_siddon_forward_runs<KP, 8>), grid, dim3(block), lds, s, vol_t, L.d_sid, sid_args(L), kmax, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_siddon_forward_runs launch");
    return CBCT_OK;
}

cbct_status cbct_launch_forward_siddon(const Level &L, const float *vol_t, float *out, hipStream_t s) {
    {
        // the run-summing kernel when its tables fit: rays in mirrored pairs, up to 256 threads
        const int npairs = (L.nv + 1) / 2;
        int npt = 1;
        while ((npairs + npt - 1) / npt > 256) npt *= 2;
        const int block = (((npairs + npt - 1) / npt + 63) / 64) * 64;
        const int kmax = L.nx + L.ny + 3;
        constexpr size_t budget = 48 * 1024;
        if (npt <= 8 && sid_runs_lds(64, L.nz, kmax, block / 64) <= budget)
            return launch_sid_runs<64>(L, vol_t, out, s, npt, block, kmax, sid_runs_lds(64, L.nz, kmax, block / 64));
        if (npt <= 8 && sid_runs_lds(32, L.nz, kmax, block / 64) <= budget)
            return launch_sid_runs<32>(L, vol_t, out, s, npt, block, kmax, sid_runs_lds(32, L.nz, kmax, block / 64));
        if (npt <= 8 && sid_runs_lds(16, L.nz, kmax, block / 64) <= budget)
            return launch_sid_runs<16>(L, vol_t, out, s, npt, block, kmax, sid_runs_lds(16, L.nz, kmax, block / 64));
    }
    const int nchunk = (L.nv + 63) / 64;
    const long items = (long)L.nviews * L.nu * nchunk;
    const long blocks = (items + 3) / 4;
    if (blocks > 0x7fffffffL) return cbct_set_error(CBCT_ERR_INVALID_ARG, "forward_siddon: grid too large");
    hipLaunchKernelGGL(k_siddon_forward, dim3((unsigned)blocks), dim3(256), 0, s, vol_t, L.d_sid, sid_args(L), nchunk,
                       out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_siddon_forward launch");
    return CBCT_OK;
}

cbct_status cbct_launch_adjoint_siddon(const Level &L, const float *proj, float *out, hipStream_t s) {
    const long blocks = (long)((L.nx + 15) / 16) * ((L.ny + 15) / 16) * ((L.nz + SID_TZ - 1) / SID_TZ);
    if (blocks > 0x7fffffffL) return cbct_set_error(CBCT_ERR_INVALID_ARG, "adjoint_siddon: grid too large");
    hipLaunchKernelGGL(k_siddon_gather, dim3((unsigned)blocks), dim3(256), 0, s, proj, L.d_sid, L.d_views, sid_args(L),
                       out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_siddon_gather launch");
    return CBCT_OK;
}
