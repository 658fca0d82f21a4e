// Per-level geometry tables of the projector pair (as the plan builds them and the P and P^T
// kernels read them) and the adjoint gather's tiling and view-group split.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

// Per (view, detector column) parameters of the column-coherent ray samples, prepared in FP64
// on the host.  Sample k of column i lies at transverse distance tau_c + k*dtau from the
// source; its voxel-index coordinates are (fx0 + k dfx, fy0 + k dfy), and detector row j
// (q_j = j - (nv-1)/2) meets it at z-index gamma_k q_j + (nz-1)/2 with gamma_k = g0 + k dg.
struct ColParams {
    float fx0, fy0;  // index coordinates of sample 0 (closest approach of the column's line to the axis)
    float dfx, dfy;  // index-coordinate step per sample
    float g0, dg;    // z cells per detector row at sample k: gamma_k = g0 + k dg  (> 0)
    float wsc, r2;   // ray step weight w_ij = wsc * sqrt(r2 + v_j^2)
    int klo, khi;    // samples whose transverse position is within one voxel of the grid (inclusive)
    float idfx, idfy; // 1/dfx, 1/dfy (0 when the step along that axis vanishes)
};
static_assert(sizeof(ColParams) == 48, "ColParams layout");

struct ViewParams {
    float cs, sn;    // cos(theta), sin(theta)
    float pad0, pad1;
};

// Per (view, detector column) line of the Siddon projector pair, prepared in FP64 on the host.
// tau is the transverse distance along the column's xy line from C, its closest approach to the
// rotation axis: the line is (cx, cy) + tau (ex, ey); the source lies at tau = -t0 and the
// detector at tau = lxy - t0 (lxy = |D - S|_xy).
struct SidCol {
    float cx, cy;    // C (mm)
    float ex, ey;    // unit direction, source to detector
    float iex, iey;  // 1/ex, 1/ey (0 when |e| <= 1e-12: the line runs parallel to those planes)
    float t0, lxy, ilxy;
    float t0lo, lxylo;  // t0 - (double)t0 and lxy - (double)lxy: the FP64 values as float pairs
    float pad;
};
static_assert(sizeof(SidCol) == 48, "SidCol layout");

// Tiling of the adjoint gather.
constexpr int ADJ_TX = 16;     // voxel columns per tile in x (lanes)
constexpr int ADJ_TY = 16;     // voxel columns per tile in y (lanes)

// Geometry the adjoint gather needs per level.
struct AdjArgs {
    int nx, ny, nz, nu, nv, nviews;
    float hx, hy, hz, pu, pv, sad, sdd;
};

// z cells per tile of the staged gather (0: depth not a multiple of 32, per-lane gather)
inline int cbct_adj_staged_tz(int nz) { return nz % 32 == 0 ? 32 : 0; }

// View groups of the staged adjoint gather (depth a multiple of 32): the views are split into
// groups (one work-group per 16 x 16 x 32 tile and group) whose partial volumes are summed in
// group order.  Small grids have few tiles, so they get about 2048 work-groups in all; large
// ones at least two groups: at 512x512x64 / 40 views two groups of 20 views (4096 work-groups,
// shorter ones, and a shorter tail) measured 1.79 against 1.94 ms per P^T including the sum.

// z cells per thread of the per-lane gather (depths that are not a multiple of 32)
inline int cbct_adj_lane_tz(int nz) {
    if (nz % 64 == 0) return 64;
    if (nz % 32 == 0) return 32;
    if (nz % 16 == 0) return 16;
    if (nz % 8 == 0) return 8;
    return nz > 32 ? 64 : nz > 16 ? 32 : nz > 8 ? 16 : 8;  // partial last tile, scalar loads
}

// The per-lane gather splits the views of small grids the same way, so that a grid of a few
// tiles still spreads over the GPU: a 16^3 volume runs 16 work-groups of one view each instead
// of one work-group walking all views.
inline int cbct_adj_vsplit(int nx, int ny, int nz, int nviews) {
    const int tz = cbct_adj_staged_tz(nz);
    if (!tz) {
        const int ltz = cbct_adj_lane_tz(nz);
        const long tiles = (long)((nx + 15) / 16) * ((ny + 15) / 16) * ((nz + ltz - 1) / ltz);
        long vs = 256 / std::max(tiles, 1L);
        vs = std::min(vs, std::min<long>(16, nviews));
        return (int)std::max(vs, 1L);
    }
    const long tiles = (long)((nx + 15) / 16) * ((ny + 15) / 16) * (nz / tz);
    long vs = std::max(2048 / std::max(tiles, 1L), 2L);
    vs = std::min(vs, std::min<long>(16, nviews));
    return (int)std::max(vs, 1L);
}

// Where the z profiles of one (view, column) live in the adjoint's workspace: samples
// k0 .. k0+nk-1 (those whose transverse position is within one voxel of the grid), nz floats each.
struct ZIndex {
    long off;  // float offset, a multiple of 32
    int k0, nk;
};
static_assert(sizeof(ZIndex) == 16, "ZIndex layout");
