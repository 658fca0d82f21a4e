// The paper's voxel-driven backprojector (Section II.C.2, Eq. 6 with the Jacobian of Eq. A7): for
// every voxel centre V and view, the line from the source through V meets the imager at
// (u*, v*) (Eq. A6 rotated to the view); the detector image T is sampled there by bilinear
// interpolation between pixel centres (zero beyond the imager) and weighted by
// L^3 / (L0 l^2) = SDD^2 l / w^3, where w is V's depth along the central ray, l = |V - S| and
// L = |P - S| = (SDD / w) l.  The sum over views is scaled by hx hy hz / (pu pv), which makes
// the operator the continuum limit of P^T, so it can replace P^T in Step 1 with the same step.
//
// One thread per voxel column segment of 16 z cells, x fastest (lanes of a wave sample
// neighbouring detector columns, which the caches serve): per view the column's u* terms are
// computed once and each cell adds its v* row pair; all views in registers, one write per voxel.
// The view's image is read through a raw buffer of its size at non-negative byte offsets: one
// address per row (the neighbouring column sits 4 bytes further; column -1 is shifted to column 0
// with its weight), rows clamped into the image with weight 0 outside it.
#include <hip/hip_runtime.h>

#include "cbct_internal.h"

namespace {

constexpr int EQ6_ZC = 16;  // z cells per thread: the view's u-side terms are shared by them

__global__ void __launch_bounds__(256)
    k_backproject_eq6(const float *__restrict__ T, const ViewParams *__restrict__ views, AdjArgs A,
                      const float *__restrict__ fbase, float kappa, float *__restrict__ out,
                      float *__restrict__ out2) {
    const long ncol = (long)A.nx * A.ny;
    const long tidg = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nzc = (A.nz + EQ6_ZC - 1) / EQ6_ZC;
    if (tidg >= ncol * nzc) return;
    const long colx = tidg % ncol;  // x fastest within a z chunk: neighbouring lanes, neighbouring columns
    const int zc = (int)(tidg / ncol);
    const int a = (int)(colx % A.nx), b = (int)(colx / A.nx);
    const int c0 = zc * EQ6_ZC;
    const float x = ((float)a - 0.5f * (float)(A.nx - 1)) * A.hx;
    const float y = ((float)b - 0.5f * (float)(A.ny - 1)) * A.hy;
    const float zc0 = ((float)c0 - 0.5f * (float)(A.nz - 1)) * A.hz;
    const float cu = 0.5f * (float)(A.nu - 1), cv = 0.5f * (float)(A.nv - 1);
    const float ipu = 1.0f / A.pu, ipv = 1.0f / A.pv;
    const float sdd2 = A.sdd * A.sdd;
    const long plane = (long)A.nu * A.nv;
    const int nu4 = A.nu * 4;
    float acc[EQ6_ZC];
#pragma unroll
    for (int q = 0; q < EQ6_ZC; q++) acc[q] = 0.0f;
    for (int view = 0; view < A.nviews; view++) {
        const ViewParams vp = views[view];
        const float w = fmaf(x, vp.cs, fmaf(y, vp.sn, A.sad));  // depth of V beyond the source
        const float t = fmaf(x, vp.sn, -y * vp.cs);             // offset along e_u
        const float iw = 1.0f / w;
        const float fu = fmaf(A.sdd * t * iw, ipu, cu);          // detector column coordinate of u*
        const float fu0 = floorf(fu);
        const int i0 = (int)fu0;
        if (i0 < -1 || i0 >= A.nu) continue;
        const float du = fu - fu0;
        const float wu0 = (i0 >= 0) ? 1.0f - du : 0.0f, wu1 = (i0 + 1 < A.nu) ? du : 0.0f;
        const float w2t2 = fmaf(w, w, t * t);
        const float wk = sdd2 * iw * iw * iw;                    // L^3/(L0 l^2) = SDD^2 l / w^3
        const float vstep = A.sdd * iw * ipv;                    // v* in rows per mm of z
        const __amdgpu_buffer_rsrc_t img = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(T + view * plane), 0, (int)(plane * 4), 0x00020000);
        // columns i0 and i0 + 1 of a row at byte offsets ob and ob + 4; i0 = -1 becomes column 0
        // carrying the weight of column i0 + 1 (the column past the last one has weight 0)
        const int ob = max(i0, 0) * 4;
        const float cw0 = i0 >= 0 ? wu0 : wu1, cw1 = i0 >= 0 ? wu1 : 0.0f;
#pragma unroll
        for (int q = 0; q < EQ6_ZC; q++) {
            const float z = fmaf((float)q, A.hz, zc0);
            const float fv = fmaf(z, vstep, cv);
            const float fv0 = floorf(fv);
            const int j0 = (int)fv0;
            const float dv = fv - fv0;
            const float wv0 = (j0 >= 0 && j0 < A.nv) ? 1.0f - dv : 0.0f;
            const float wv1 = (j0 + 1 >= 0 && j0 + 1 < A.nv) ? dv : 0.0f;
            const int o0 = min(max(j0, 0), A.nv - 1) * nu4 + ob, o1 = min(max(j0 + 1, 0), A.nv - 1) * nu4 + ob;
            const float r00 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(img, o0, 0, 0));
            const float r01 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(img, o0 + 4, 0, 0));
            const float r10 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(img, o1, 0, 0));
            const float r11 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(img, o1 + 4, 0, 0));
            const float s = fmaf(wv0, fmaf(cw0, r00, cw1 * r01), wv1 * fmaf(cw0, r10, cw1 * r11));
            const float l = __builtin_amdgcn_sqrtf(fmaf(z, z, w2t2));
            acc[q] = fmaf(wk * l, s, acc[q]);
        }
    }
    const float scale = A.hx * A.hy * A.hz * ipu * ipv;
#pragma unroll
    for (int q = 0; q < EQ6_ZC; q++) {
        const int c = c0 + q;
        if (c < A.nz) {
            const long idx = ((long)c * A.ny + b) * A.nx + a;
            const float v = acc[q] * scale;
            const float o = fbase ? fmaf(-kappa, v, fbase[idx]) : v;
            out[idx] = o;
            if (out2) out2[idx] = o;
        }
    }
}

}  // namespace

cbct_status cbct_launch_backproject_eq6(const Level &L, const float *proj, const float *fbase, float kappa, float *out,
                                        hipStream_t s, float *out2) {
    const long n = (long)L.nx * L.ny * ((L.nz + EQ6_ZC - 1) / EQ6_ZC);
    hipLaunchKernelGGL(k_backproject_eq6, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, proj, L.d_views, L.adj,
                       fbase, kappa, out, out2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cbct_hip_error(e, "k_backproject_eq6 launch");
    return CBCT_OK;
}
