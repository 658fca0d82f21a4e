// Plans: FP64 geometry of every multigrid level, uploaded as FP32 kernel tables; status
// plumbing; the forward/adjoint entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "cbct_internal.h"

static thread_local char g_err[512] = "";

cbct_status cbct_set_error(cbct_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

cbct_status cbct_hip_error(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory) return cbct_set_error(CBCT_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
    return cbct_set_error(CBCT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char *cbct_last_error(void) { return g_err; }

extern "C" const char *cbct_status_string(cbct_status s) {
    switch (s) {
    case CBCT_OK: return "CBCT_OK";
    case CBCT_ERR_INVALID_ARG: return "CBCT_ERR_INVALID_ARG";
    case CBCT_ERR_OUT_OF_MEMORY: return "CBCT_ERR_OUT_OF_MEMORY";
    case CBCT_ERR_BUDGET: return "CBCT_ERR_BUDGET";
    case CBCT_ERR_HIP: return "CBCT_ERR_HIP";
    case CBCT_ERR_NONFINITE: return "CBCT_ERR_NONFINITE";
    case CBCT_ERR_NOT_FOUND: return "CBCT_ERR_NOT_FOUND";
    case CBCT_ERR_INTERNAL: return "CBCT_ERR_INTERNAL";
    }
    return "CBCT_ERR_UNKNOWN";
}

// Samples k (relative to the closest approach) whose index coordinate f0 + k df lies in
// (-1, n): the open interval where the zero-extended interpolant can be non-zero, widened by
// one sample on each side.
static void sample_range_1d(double f0, double df, int n, double &lo, double &hi) {
    if (std::fabs(df) < 1e-12) {
        if (f0 > -1.0 && f0 < n) {
            lo = -1e18;
            hi = 1e18;
        } else {
            lo = 1e18;
            hi = -1e18;
        }
        return;
    }
    double a = (-1.0 - f0) / df, b = ((double)n - f0) / df;
    lo = std::min(a, b);
    hi = std::max(a, b);
}

static cbct_status build_level(const cbct_geometry_desc *g, int l, int bin, Level &L) {
    const int f = 1 << l;
    L.nx = g->nx / f;
    L.ny = g->ny / f;
    L.nz = g->nz / f;
    L.hx = g->hx * f;
    L.hy = g->hy * f;
    L.hz = g->hz * f;
    L.nu = bin ? g->nu / f : g->nu;
    L.nv = bin ? g->nv / f : g->nv;
    L.pu = bin ? g->pu * f : g->pu;
    L.pv = bin ? g->pv * f : g->pv;
    L.sad = g->sad;
    L.sdd = g->sdd;
    L.nviews = g->n_views;
    double rho = g->sample_ratio > 0.0 ? g->sample_ratio : 1.0;
    L.dtau = rho * std::min(g->hx, g->hy) * f;
    L.angles.resize(L.nviews);
    for (int v = 0; v < L.nviews; v++)
        L.angles[v] = g->angles ? g->angles[v] : 2.0 * M_PI * (double)v / (double)L.nviews;

    std::vector<ColParams> cols((size_t)L.nviews * L.nu);
    std::vector<SidCol> sid((size_t)L.nviews * L.nu);
    std::vector<ViewParams> views(L.nviews);
    double smax = 0.0;
    for (int v = 0; v < L.nviews; v++) {
        const double cs = std::cos(L.angles[v]), sn = std::sin(L.angles[v]);
        views[v] = ViewParams{(float)cs, (float)sn, 0.f, 0.f};
        // e_w = (cs, sn), e_u = (sn, -cs)
        for (int i = 0; i < L.nu; i++) {
            const double u = (i - 0.5 * (L.nu - 1)) * L.pu;
            const double r2 = L.sdd * L.sdd + u * u, r = std::sqrt(r2);
            const double mx = (L.sdd * cs + u * sn) / r, my = (L.sdd * sn - u * cs) / r;
            // closest approach of the column's transverse line to the axis, cancellation-free:
            // C = (sad / r^2) (sdd u e_u - u^2 e_w)
            const double cx = L.sad / r2 * (L.sdd * u * sn - u * u * cs);
            const double cy = L.sad / r2 * (-L.sdd * u * cs - u * u * sn);
            const double tau_c = L.sad * L.sdd / r;
            SidCol &sc = sid[(size_t)v * L.nu + i];
            sc = SidCol{};
            sc.cx = (float)cx;
            sc.cy = (float)cy;
            sc.ex = (float)mx;
            sc.ey = (float)my;
            sc.iex = std::fabs(mx) > 1e-12 ? (float)(1.0 / mx) : 0.0f;
            sc.iey = std::fabs(my) > 1e-12 ? (float)(1.0 / my) : 0.0f;
            sc.t0 = (float)tau_c;
            sc.lxy = (float)r;
            sc.t0lo = (float)(tau_c - (double)sc.t0);
            sc.lxylo = (float)(r - (double)sc.lxy);
            sc.ilxy = (float)(1.0 / r);
            ColParams &c = cols[(size_t)v * L.nu + i];
            const double fx0 = cx / L.hx + 0.5 * (L.nx - 1), fy0 = cy / L.hy + 0.5 * (L.ny - 1);
            const double dfx = L.dtau * mx / L.hx, dfy = L.dtau * my / L.hy;
            double lx, hx_, ly, hy_;
            sample_range_1d(fx0, dfx, L.nx, lx, hx_);
            sample_range_1d(fy0, dfy, L.ny, ly, hy_);
            double lo = std::max(lx, ly), hi = std::min(hx_, hy_);
            int klo = 1, khi = 0;
            if (lo < hi) {
                klo = (int)std::floor(lo) - 1;
                khi = (int)std::ceil(hi) + 1;
            }
            c.fx0 = (float)fx0;
            c.fy0 = (float)fy0;
            c.dfx = (float)dfx;
            c.dfy = (float)dfy;
            c.g0 = (float)(tau_c * L.pv / (r * L.hz));
            c.dg = (float)(L.dtau * L.pv / (r * L.hz));
            c.wsc = (float)(L.dtau / r);
            c.r2 = (float)r2;
            c.klo = klo;
            c.khi = khi;
            c.idfx = std::fabs(dfx) > 1e-12 ? (float)(1.0 / dfx) : 0.0f;
            c.idfy = std::fabs(dfy) > 1e-12 ? (float)(1.0 / dfy) : 0.0f;
            if (khi >= klo) {
                // up to one chunk (<= 64 samples) is appended below to fill whole chunks
                double gmax = (tau_c + (khi + 64) * L.dtau) * L.pv / (r * L.hz);
                smax = std::max(smax, gmax * 0.5 * (L.nv - 1));
            }
        }
    }
    // forward tables: z index s in [(nz-1)/2 - smax, (nz-1)/2 + smax] must stay inside the
    // padded table, whose real cells sit at offset pad+1
    const double beta = 0.5 * (L.nz - 1);
    L.fwd_pad = std::max(0, (int)std::ceil(smax - beta)) + 1;
    L.fwd_tw = L.nz + 2 * L.fwd_pad + 3;
    L.fwd_kc = ((size_t)L.fwd_tw * 65 * 4 <= 56 * 1024) ? 32 : 16;
    // the run-summing projector (no z padding needed; 32-bit byte offsets into the volume)
    L.fwd_kr = L.nvox() * 4 < (1L << 31) ? cbct_forward_run_chunk(L.nz, cbct_forward_runs_block(L.nv, nullptr) / 64) : 0;
    if (L.fwd_kr == 0 && (size_t)L.fwd_tw * (2 * L.fwd_kc + 1) * 4 > 60 * 1024)
        return cbct_set_error(CBCT_ERR_INVALID_ARG,
                              "level %d: cone too wide for the projector tables (%d z cells)", l, L.fwd_tw);
    // adjoint profile workspace: the samples of each column inside the grid's support
    std::vector<ZIndex> zix(cols.size());
    long zoff = 0;
    for (size_t q = 0; q < cols.size(); q++) {
        const int nk = std::max(cols[q].khi - cols[q].klo + 1, 0);
        zix[q] = ZIndex{zoff, cols[q].klo, nk};
        L.zk_max = std::max(L.zk_max, nk);
        zoff += ((long)nk * L.nz + 31) & ~31L;  // column blocks start on 128-byte lines
    }
    L.adj_vsplit = cbct_adj_vsplit(L.nx, L.ny, L.nz, L.nviews);
    if (L.adj_vsplit > 1) {
        L.adj_part_off = (zoff + 63) & ~63L;
        zoff = L.adj_part_off + (long)L.adj_vsplit * L.nvox();
    }
    L.z_floats = std::max(zoff, 4L);
    AdjArgs &A = L.adj;
    A.nx = L.nx; A.ny = L.ny; A.nz = L.nz; A.nu = L.nu; A.nv = L.nv; A.nviews = L.nviews;
    A.hx = (float)L.hx; A.hy = (float)L.hy; A.hz = (float)L.hz; A.pu = (float)L.pu; A.pv = (float)L.pv;
    A.sad = (float)L.sad; A.sdd = (float)L.sdd;
    // whole chunks for the projector: extend every sample range to a multiple of the chunk of the
    // projector this level runs (the run-summing one when it fits, else the per-sample one; the
    // extra samples lie beyond the grid, where all interpolation weights vanish)
    const int kpad = L.fwd_kr > 0 ? L.fwd_kr : L.fwd_kc;
    for (auto &c : cols)
        if (c.khi >= c.klo) c.khi = c.klo + ((c.khi - c.klo + kpad) / kpad) * kpad - 1;

    if (std::getenv("CBCT_PLAN_REPORT"))
        std::fprintf(stderr,
                     "[cbct plan] level %d: %dx%dx%d voxels, %d views %dx%d; fwd pad %d kc %d kr %d lds %zu; "
                     "adjoint profiles %.1f MB\n",
                     l, L.nx, L.ny, L.nz, L.nviews, L.nu, L.nv, L.fwd_pad, L.fwd_kc, L.fwd_kr,
                     (size_t)L.fwd_tw * (2 * L.fwd_kc + 1) * 4, 4e-6 * (double)L.z_floats);
    CBCT_HIP(hipMalloc((void **)&L.d_cols, sizeof(ColParams) * cols.size()));
    CBCT_HIP(hipMalloc((void **)&L.d_views, sizeof(ViewParams) * views.size()));
    CBCT_HIP(hipMemcpy(L.d_cols, cols.data(), sizeof(ColParams) * cols.size(), hipMemcpyHostToDevice));
    CBCT_HIP(hipMemcpy(L.d_views, views.data(), sizeof(ViewParams) * views.size(), hipMemcpyHostToDevice));
    CBCT_HIP(hipMalloc((void **)&L.d_sid, sizeof(SidCol) * sid.size()));
    CBCT_HIP(hipMemcpy(L.d_sid, sid.data(), sizeof(SidCol) * sid.size(), hipMemcpyHostToDevice));
    CBCT_HIP(hipMalloc((void **)&L.d_zix, sizeof(ZIndex) * zix.size()));
    CBCT_HIP(hipMemcpy(L.d_zix, zix.data(), sizeof(ZIndex) * zix.size(), hipMemcpyHostToDevice));
    return CBCT_OK;
}

extern "C" cbct_status cbct_context_create(int hip_device, cbct_context **out) {
    if (!out) return cbct_set_error(CBCT_ERR_INVALID_ARG, "context_create: NULL out");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "context_create: no HIP device (%s)", hipGetErrorString(e));
    }
    if (hip_device < 0 || hip_device >= n)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "context_create: device %d not in [0, %d)", hip_device, n);
    hipDeviceProp_t prop;
    CBCT_HIP(hipGetDeviceProperties(&prop, hip_device));
    // the library's code objects are built for gfx950 only
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "context_create: device %d is %s, the library is built for gfx950",
                              hip_device, prop.gcnArchName);
    {
        // per device, once: the address of the no-allocation entry point's scratch array
        DeviceGuard dg(hip_device);
        cbct_status st = cbct_noalloc_scratch_init(hip_device);
        if (st) return st;
    }
    cbct_context *c = new (std::nothrow) cbct_context();
    if (!c) return cbct_set_error(CBCT_ERR_OUT_OF_MEMORY, "context_create: host allocation");
    c->device = hip_device;
    c->total_mem = prop.totalGlobalMem;
    std::snprintf(c->arch, sizeof(c->arch), "%s", prop.gcnArchName);
    *out = c;
    return CBCT_OK;
}

extern "C" void cbct_context_destroy(cbct_context *ctx) { delete ctx; }

extern "C" cbct_status cbct_context_device(const cbct_context *ctx, int *hip_device) {
    if (!ctx || !hip_device) return cbct_set_error(CBCT_ERR_INVALID_ARG, "context_device: NULL argument");
    *hip_device = ctx->device;
    return CBCT_OK;
}

extern "C" cbct_status cbct_plan_create(cbct_context *ctx, const cbct_geometry_desc *g, int levels,
                                        int bin_detector, cbct_plan **out) {
    if (!g || !out) return cbct_set_error(CBCT_ERR_INVALID_ARG, "plan_create: NULL argument");
    *out = nullptr;
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || g->nu <= 0 || g->nv <= 0 || g->n_views <= 0)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "plan_create: sizes must be positive");
    if (!(g->hx > 0 && g->hy > 0 && g->hz > 0 && g->pu > 0 && g->pv > 0))
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "plan_create: pitches must be positive");
    if (levels < 1 || levels > 8) return cbct_set_error(CBCT_ERR_INVALID_ARG, "plan_create: levels must be 1..8");
    const double half_diag = 0.5 * std::sqrt(std::pow((g->nx + 2) * g->hx, 2) + std::pow((g->ny + 2) * g->hy, 2));
    if (!(g->sad > half_diag) || !(g->sdd > g->sad))
        return cbct_set_error(CBCT_ERR_INVALID_ARG,
                              "plan_create: need sad > half the grid diagonal (%.1f mm) and sdd > sad", half_diag);
    const int f = 1 << (levels - 1);
    if (g->nx % f || g->ny % f || g->nz % f)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "plan_create: volume dims not divisible by 2^(levels-1) = %d", f);
    if (bin_detector && (g->nu % f || g->nv % f))
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "plan_create: detector dims not divisible by %d", f);
    if ((long)g->nx * g->ny * g->nz > (1L << 31) - 1 || (long)g->n_views * g->nu * g->nv > (1L << 31) - 1)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "plan_create: more than 2^31 voxels or detector samples");
    if (g->nv > 2048 || g->nu > 16384)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "plan_create: detector larger than 16384 x 2048");

    if (!ctx) return cbct_set_error(CBCT_ERR_INVALID_ARG, "plan_create: NULL context");
    cbct_plan *p = new (std::nothrow) cbct_plan();
    if (!p) return cbct_set_error(CBCT_ERR_OUT_OF_MEMORY, "plan_create: host allocation");
    DeviceGuard dg(ctx->device);
    p->device = ctx->device;
    p->levels = levels;
    p->bin_detector = bin_detector ? 1 : 0;
    p->lv.resize(levels);
    for (int l = 0; l < levels; l++) {
        cbct_status s = build_level(g, l, p->bin_detector, p->lv[l]);
        if (s != CBCT_OK) {
            cbct_plan_destroy(p);
            return s;
        }
    }
    *out = p;
    return CBCT_OK;
}

extern "C" void cbct_plan_destroy(cbct_plan *p) {
    if (!p) return;
    DeviceGuard dg(p->device);
    for (auto &L : p->lv) {
        if (L.d_cols) hipFree(L.d_cols);
        if (L.d_views) hipFree(L.d_views);
        if (L.d_zix) hipFree(L.d_zix);
        if (L.d_sid) hipFree(L.d_sid);
    }
    delete p;
}

static cbct_status check_level(const cbct_plan *p, int level, const char *who) {
    if (!p) return cbct_set_error(CBCT_ERR_INVALID_ARG, "%s: NULL plan", who);
    if (level < 0 || level >= p->levels)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "%s: level %d out of range [0, %d)", who, level, p->levels);
    return CBCT_OK;
}

extern "C" cbct_status cbct_plan_level_dims(const cbct_plan *p, int level, int out[6]) {
    cbct_status s = check_level(p, level, "plan_level_dims");
    if (s) return s;
    if (!out) return cbct_set_error(CBCT_ERR_INVALID_ARG, "plan_level_dims: NULL out");
    const Level &L = p->lv[level];
    out[0] = L.nx;
    out[1] = L.ny;
    out[2] = L.nz;
    out[3] = L.nu;
    out[4] = L.nv;
    out[5] = L.nviews;
    return CBCT_OK;
}

extern "C" cbct_status cbct_forward_workspace_size(const cbct_plan *p, int level, size_t *bytes) {
    cbct_status s = check_level(p, level, "forward_workspace_size");
    if (s) return s;
    if (!bytes) return cbct_set_error(CBCT_ERR_INVALID_ARG, "forward_workspace_size: NULL out");
    *bytes = (size_t)p->lv[level].nvox() * sizeof(float);
    return CBCT_OK;
}

extern "C" cbct_status cbct_forward(const cbct_plan *p, int level, const float *d_vol, float *d_proj, void *d_ws,
                                    size_t ws_bytes, cbct_stream_t stream) {
    cbct_status s = check_level(p, level, "forward");
    if (s) return s;
    DeviceGuard dg(p->device);
    if (!d_vol || !d_proj || !d_ws) return cbct_set_error(CBCT_ERR_INVALID_ARG, "forward: NULL pointer");
    const Level &L = p->lv[level];
    if (ws_bytes < (size_t)L.nvox() * sizeof(float))
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "forward: workspace %zu < %zu bytes", ws_bytes,
                              (size_t)L.nvox() * sizeof(float));
    if (((uintptr_t)d_ws & 15) != 0)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "forward: workspace must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    s = cbct_launch_to_columns(L, d_vol, (float *)d_ws, st);
    if (s) return s;
    return cbct_launch_forward(L, (const float *)d_ws, nullptr, d_proj, nullptr, st);
}

extern "C" cbct_status cbct_adjoint_workspace_size(const cbct_plan *p, int level, size_t *bytes) {
    cbct_status s = check_level(p, level, "adjoint_workspace_size");
    if (s) return s;
    if (!bytes) return cbct_set_error(CBCT_ERR_INVALID_ARG, "adjoint_workspace_size: NULL out");
    *bytes = (size_t)p->lv[level].z_floats * sizeof(float);
    return CBCT_OK;
}

extern "C" cbct_status cbct_adjoint(const cbct_plan *p, int level, const float *d_proj, float *d_vol, void *d_ws,
                                    size_t ws_bytes, cbct_stream_t stream) {
    cbct_status s = check_level(p, level, "adjoint");
    if (s) return s;
    DeviceGuard dg(p->device);
    if (!d_proj || !d_vol || !d_ws) return cbct_set_error(CBCT_ERR_INVALID_ARG, "adjoint: NULL pointer");
    const Level &L = p->lv[level];
    if (ws_bytes < (size_t)L.z_floats * sizeof(float))
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "adjoint: workspace %zu < %zu bytes", ws_bytes,
                              (size_t)L.z_floats * sizeof(float));
    if (((uintptr_t)d_ws & 15) != 0)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "adjoint: workspace must be 16-byte aligned");
    return cbct_launch_adjoint(L, d_proj, nullptr, 0.0f, d_vol, (float *)d_ws, (hipStream_t)stream);
}

extern "C" cbct_status cbct_forward_columns(const cbct_plan *p, int level, const float *d_vol_cols, float *d_proj,
                                            cbct_stream_t stream) {
    cbct_status s = check_level(p, level, "forward_columns");
    if (s) return s;
    DeviceGuard dg(p->device);
    if (!d_vol_cols || !d_proj) return cbct_set_error(CBCT_ERR_INVALID_ARG, "forward_columns: NULL pointer");
    if (((uintptr_t)d_vol_cols & 15) != 0)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "forward_columns: volume must be 16-byte aligned");
    return cbct_launch_forward(p->lv[level], d_vol_cols, nullptr, d_proj, nullptr, (hipStream_t)stream);
}

extern "C" cbct_status cbct_forward_siddon(const cbct_plan *p, int level, const float *d_vol, float *d_proj,
                                           void *d_ws, size_t ws_bytes, cbct_stream_t stream) {
    cbct_status s = check_level(p, level, "forward_siddon");
    if (s) return s;
    DeviceGuard dg(p->device);
    if (!d_vol || !d_proj || !d_ws) return cbct_set_error(CBCT_ERR_INVALID_ARG, "forward_siddon: NULL pointer");
    const Level &L = p->lv[level];
    if (ws_bytes < (size_t)L.nvox() * sizeof(float))
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "forward_siddon: workspace %zu < %zu bytes", ws_bytes,
                              (size_t)L.nvox() * sizeof(float));
    hipStream_t st = (hipStream_t)stream;
    s = cbct_launch_to_columns(L, d_vol, (float *)d_ws, st);
    if (s) return s;
    return cbct_launch_forward_siddon(L, (const float *)d_ws, nullptr, d_proj, nullptr, st);
}

extern "C" cbct_status cbct_adjoint_siddon_workspace_size(const cbct_plan *p, int level, size_t *bytes) {
    cbct_status s = check_level(p, level, "adjoint_siddon_workspace_size");
    if (s) return s;
    if (!bytes) return cbct_set_error(CBCT_ERR_INVALID_ARG, "adjoint_siddon_workspace_size: NULL out");
    *bytes = cbct_adjoint_siddon_ws_bytes(p->lv[level]);
    return CBCT_OK;
}

extern "C" cbct_status cbct_adjoint_siddon(const cbct_plan *p, int level, const float *d_proj, float *d_vol,
                                           void *d_ws, size_t ws_bytes, cbct_stream_t stream) {
    cbct_status s = check_level(p, level, "adjoint_siddon");
    if (s) return s;
    DeviceGuard dg(p->device);
    if (!d_proj || !d_vol || !d_ws) return cbct_set_error(CBCT_ERR_INVALID_ARG, "adjoint_siddon: NULL pointer");
    const Level &L = p->lv[level];
    const size_t need = cbct_adjoint_siddon_ws_bytes(L);
    if (ws_bytes < need)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "adjoint_siddon: workspace %zu < %zu bytes", ws_bytes, need);
    if (((uintptr_t)d_ws & 255) != 0)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "adjoint_siddon: workspace must be 256-byte aligned");
    return cbct_launch_adjoint_siddon(L, d_proj, nullptr, 0.0f, d_vol, d_ws, (hipStream_t)stream);
}

extern "C" cbct_status cbct_backproject_eq6(const cbct_plan *p, int level, const float *d_proj, float *d_vol,
                                            cbct_stream_t stream) {
    cbct_status s = check_level(p, level, "backproject_eq6");
    if (s) return s;
    DeviceGuard dg(p->device);
    if (!d_proj || !d_vol) return cbct_set_error(CBCT_ERR_INVALID_ARG, "backproject_eq6: NULL pointer");
    return cbct_launch_backproject_eq6(p->lv[level], d_proj, nullptr, 0.0f, d_vol, (hipStream_t)stream);
}
