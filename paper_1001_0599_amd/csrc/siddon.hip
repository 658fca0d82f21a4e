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

SidArgs sid_args(const Level &L) {
    SidArgs A;
    A.nx = L.nx; A.ny = L.ny; A.nz = L.nz; A.nu = L.nu; A.nv = L.nv; A.nviews = L.nviews;
    A.hx = (float)L.hx; A.hy = (float)L.hy; A.hz = (float)L.hz; A.pu = (float)L.pu; A.pv = (float)L.pv;
    A.sad = (float)L.sad; A.sdd = (float)L.sdd;
    return A;
}

}  // namespace

cbct_status cbct_launch_forward_siddon(const Level &L, const float *vol_t, float *out, hipStream_t s) {
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
