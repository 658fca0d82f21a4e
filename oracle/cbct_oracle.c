/*
 * CPU oracle: TV-regularised cone-beam CT reconstruction by forward-backward
 * splitting (Jia, Lou, Lewis, Li, Gu, Men, Song, Jiang: "GPU-based fast low-dose
 * cone beam CT reconstruction via total variation").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * helper with the GPU library, and it is deliberately plain and slow: double
 * precision everywhere, one loop per definition, no blocking or reordering.
 *
 * Readings of points the paper leaves open:
 *   - P (Eq. 1) is the ray integral of the zero-extended trilinear interpolant of
 *     the voxel grid, taken as a Riemann sum with a fixed step: every ray of one
 *     detector column visits the points whose transverse (xy) distance from the
 *     source is tau_c + k*dtau, where tau_c is that column's closest approach to
 *     the rotation axis.  The 3-D step of the sum is dtau*|D-S|/|D-S|_xy.
 *   - P^T is the exact matrix transpose of that P (Section II.C.2, first
 *     paragraph: the gradient of E2 is P^T(P f - Y) up to constants).
 *   - The weight mu on E2 in Eq. (2) becomes lambda = 1/mu on the TV term; the
 *     1/V and 1/(N_theta A) normalisations are means over voxels and detector
 *     samples:  E(f) = D(f) + lambda R(f),  D = mean((Pf-Y)^2),
 *     R = mean(sqrt(|grad f|^2 + eps^2)).
 *   - Boundary conditions (Section II.B, last paragraph): forward differences;
 *     the ghost beyond the last x and y sample is 0, the ghost beyond the last z
 *     plane is a copy of that plane.
 *   - Algorithm A1 with step t = mu/beta = 1/(lambda beta); by default t = 1/L with
 *     L the Schur bound of the gradient's Lipschitz constant.
 *   - Step 2 (ROF) by gradient descent with the Armijo rule of Eq. (5), c = 0.01,
 *     alpha = 0.6, eps = 0.1 %, initial step t, at most 50 iterations and 30
 *     backtracks, started from u = g.
 *   - Siddon's ray tracing (Section II.C.2; also the paper's data simulator, Section III.A)
 *     as an alternative P: each voxel is constant on its cube, and a ray's value is the sum
 *     over voxels of (length of S->D inside the cube) x voxel value.  The pieces come from the
 *     sorted parameters at which the segment crosses the grid planes; a piece's voxel is the
 *     one holding its midpoint (cubes half-open on their upper faces: a ray in a face plane
 *     belongs to the cube above it).  Its transpose is the exact matrix transpose.  Algorithm A1 can
 *     run with either pair (params.projector): the data term, the Schur bound and Step 1 then use it.
 *   - Multigrid (Section II.C.3): coarse-to-fine levels, dims halved per level
 *     over the same box, detector binned 2x2 per level, cell-centred trilinear
 *     prolongation (3/4, 1/4 per axis, clamped), restriction = (1/8) Prol^T.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int nx, ny, nz;
    double hx, hy, hz;
    int nu, nv;
    double pu, pv;
    double sad, sdd;
    int nviews;
    const double *angles; /* NULL: 2*pi*k/nviews */
    double dtau;          /* transverse sample spacing of P (mm) */
} og_geom;

typedef struct {
    double lambda;        /* TV weight (1/mu of Eq. 2) */
    double step;          /* t; <= 0: Schur bound per level */
    double tv_eps;        /* smoothing of |grad f| (1/mm^2) */
    double armijo_c;      /* c of Eq. 5 */
    double backtrack;     /* alpha of Eq. 5 */
    double rof_tol;       /* relative-decrease stop of Step 2 */
    int rof_max_iter;
    int rof_max_backtrack;
    int step1_eq6;        /* 1: Step 1 uses the Eq. 6 backprojector instead of the exact P^T */
    double conv_tol;      /* > 0: a level stops once |E(f_k) - E(f_k-1)| <= conv_tol E(f_k-1) (k >= 1);
                           * its iteration count is then the upper bound */
    int projector;        /* 0: the trilinear ray sum P and its transpose; 1: Siddon's exact path and its
                           * transpose (data term, Schur bound and Step 1) */
} og_params;

typedef struct {
    int *trace;           /* 4 ints per ROF iteration: level, outer, inner, m (m = -1: no Armijo step) */
    int trace_cap;        /* capacity in records */
    int trace_len;        /* out: records produced (may exceed trace_cap; extra ones dropped) */
    double *rof_e;        /* 3 doubles per record: E0, trial energy at the last tested step, G */
    double *energy;       /* per level (coarsest first): E(f_k), k = 0..iters */
    int energy_cap;
    int energy_len;
    double t_used[16];    /* out: t per level (index = level) */
} og_stats;

/* ---- test hook ---------------------------------------------------------------------
 * A non-zero fault plants one deliberate mistake; the pin tests must catch every one. */
static int og_fault = 0;
void orc_set_fault(int k) { og_fault = k; }

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------------- */
/* Geometry (Eq. 1, Fig. 1, Appendix Eqs. A2 and A6 at theta = 0, rotated about z).   */
/* ---------------------------------------------------------------------------------- */
static double og_angle(const og_geom *g, int view) {
    if (g->angles) return g->angles[view];
    return 2.0 * M_PI * (double)view / (double)g->nviews;
}

static long og_nvox(const og_geom *g) { return (long)g->nx * g->ny * g->nz; }
static long og_nray(const og_geom *g) { return (long)g->nviews * g->nv * g->nu; }

typedef struct {
    double S[3];   /* source */
    double dir[3]; /* (D - S) / |D - S|_xy : moves one mm per mm of transverse travel */
    double tau_c;  /* transverse distance from S to the closest approach of the axis */
    double w;      /* 3-D length of one sample step */
} og_ray;

static void og_ray_setup(const og_geom *g, int view, int i, int j, og_ray *ray) {
    double th = og_angle(g, view);
    double ew[3] = {cos(th), sin(th), 0.0};
    double eu[3] = {sin(th), -cos(th), 0.0};
    if (og_fault == 2) { eu[0] = -eu[0]; eu[1] = -eu[1]; }
    double ev[3] = {0.0, 0.0, 1.0};
    double u = (i - 0.5 * (g->nu - 1)) * g->pu;
    double v = (j - 0.5 * (g->nv - 1)) * g->pv;
    double S[3], D[3], d[3];
    for (int q = 0; q < 3; q++) {
        S[q] = -g->sad * ew[q];
        D[q] = S[q] + g->sdd * ew[q] + u * eu[q] + v * ev[q];
        d[q] = D[q] - S[q];
    }
    double r = sqrt(d[0] * d[0] + d[1] * d[1]);
    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int q = 0; q < 3; q++) {
        ray->S[q] = S[q];
        ray->dir[q] = d[q] / r;
    }
    if (og_fault == 3) ray->dir[2] = v / g->sdd; /* z slope of a parallel beam */
    /* closest approach of the transverse line S + tau*dir_xy to the axis */
    ray->tau_c = -(S[0] * ray->dir[0] + S[1] * ray->dir[1]);
    ray->w = (og_fault == 1) ? g->dtau : g->dtau * len / r;
}

/* half-width (in samples) of a sample window that contains every sample whose
 * position lies within one voxel of the grid (where the interpolant can be non-zero) */
static int og_sample_halfwidth(const og_geom *g) {
    double ex = 0.5 * (g->nx + 1) * g->hx, ey = 0.5 * (g->ny + 1) * g->hy;
    return (int)ceil(sqrt(ex * ex + ey * ey) / g->dtau) + 1;
}

static double og_hat(double s) {
    double a = fabs(s);
    return a < 1.0 ? 1.0 - a : 0.0;
}

/* continuous index coordinates of a point: voxel centres at integers */
static void og_index_coords(const og_geom *g, const double p[3], double q[3]) {
    double off = (og_fault == 11) ? 0.5 : 0.0;
    q[0] = p[0] / g->hx + 0.5 * (g->nx - 1) + off;
    q[1] = p[1] / g->hy + 0.5 * (g->ny - 1);
    q[2] = p[2] / g->hz + 0.5 * (g->nz - 1);
}

/* zero-extended trilinear interpolant f~(p) = sum_abc f_abc hat(.)hat(.)hat(.) */
static double og_interp(const og_geom *g, const double *f, const double p[3]) {
    double q[3];
    og_index_coords(g, p, q);
    int a0 = (int)floor(q[0]), b0 = (int)floor(q[1]), c0 = (int)floor(q[2]);
    double sum = 0.0;
    for (int c = c0; c <= c0 + 1; c++) {
        if (c < 0 || c >= g->nz) continue;
        double wz = og_hat(q[2] - c);
        for (int b = b0; b <= b0 + 1; b++) {
            if (b < 0 || b >= g->ny) continue;
            double wy = og_hat(q[1] - b);
            for (int a = a0; a <= a0 + 1; a++) {
                if (a < 0 || a >= g->nx) continue;
                sum += f[((long)c * g->ny + b) * g->nx + a] * og_hat(q[0] - a) * wy * wz;
            }
        }
    }
    return sum;
}

/* transpose of og_interp: acc_abc += val * hat(.)hat(.)hat(.) */
static void og_spread(const og_geom *g, double *acc, const double p[3], double val) {
    double q[3];
    og_index_coords(g, p, q);
    int a0 = (int)floor(q[0]), b0 = (int)floor(q[1]), c0 = (int)floor(q[2]);
    for (int c = c0; c <= c0 + 1; c++) {
        if (c < 0 || c >= g->nz) continue;
        double wz = (og_fault == 4) ? og_hat(q[2] - c0) : og_hat(q[2] - c);
        for (int b = b0; b <= b0 + 1; b++) {
            if (b < 0 || b >= g->ny) continue;
            double wy = og_hat(q[1] - b);
            for (int a = a0; a <= a0 + 1; a++) {
                if (a < 0 || a >= g->nx) continue;
                acc[((long)c * g->ny + b) * g->nx + a] += val * og_hat(q[0] - a) * wy * wz;
            }
        }
    }
}

static void og_sample_point(const og_ray *ray, double tau, double p[3]) {
    for (int q = 0; q < 3; q++) p[q] = ray->S[q] + tau * ray->dir[q];
}

static double og_ray_integral(const og_geom *g, const double *f, int view, int i, int j) {
    og_ray ray;
    og_ray_setup(g, view, i, j, &ray);
    int K = og_sample_halfwidth(g);
    double acc = 0.0, p[3];
    for (int k = -K; k <= K; k++) {
        og_sample_point(&ray, ray.tau_c + k * g->dtau, p);
        acc += og_interp(g, f, p);
    }
    return ray.w * acc;
}

/* P: y[view][j][i] = ray integral (Eq. 1) through the interpolated volume */
void orc_forward(const og_geom *g, const double *f, double *y) {
    long nray = og_nray(g);
#pragma omp parallel for schedule(dynamic, 64)
    for (long r = 0; r < nray; r++) {
        int i = (int)(r % g->nu);
        int j = (int)((r / g->nu) % g->nv);
        int view = (int)(r / ((long)g->nu * g->nv));
        y[r] = og_ray_integral(g, f, view, i, j);
    }
}

/* ---------------------------------------------------------------------------------- */
/* Siddon's exact radiological path (the paper's projector and data simulator,        */
/* Section II.C.2): the ray integral of the piecewise-constant volume, i.e. the sum    */
/* over voxels of the ray's length inside the voxel's cube times the voxel's value.    */
/* The plain method: every parameter alpha in (0, 1) where the segment S->D crosses a  */
/* grid plane, sorted; each piece between consecutive parameters lies in the voxel     */
/* that contains its midpoint.                                                         */
/* ---------------------------------------------------------------------------------- */
static void og_ray_ends(const og_geom *g, int view, int i, int j, double S[3], double D[3]) {
    double th = og_angle(g, view);
    double ew[3] = {cos(th), sin(th), 0.0}, eu[3] = {sin(th), -cos(th), 0.0};
    double u = (i - 0.5 * (g->nu - 1)) * g->pu, v = (j - 0.5 * (g->nv - 1)) * g->pv;
    for (int q = 0; q < 3; q++) {
        S[q] = -g->sad * ew[q];
        D[q] = S[q] + g->sdd * ew[q] + u * eu[q] + (q == 2 ? v : 0.0);
    }
}

static int og_cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* the ray's pieces: alpha breakpoints (sorted, 0 and 1 included) into buf, count returned */
static int og_siddon_alphas(const og_geom *g, const double S[3], const double D[3], double *buf) {
    const int n[3] = {g->nx, g->ny, g->nz};
    const double h[3] = {g->hx, g->hy, g->hz};
    int m = 0;
    buf[m++] = 0.0;
    buf[m++] = 1.0;
    for (int q = 0; q < 3; q++) {
        double dq = D[q] - S[q];
        if (dq == 0.0 || (og_fault == 13 && q == 2)) continue;
        for (int p = 0; p <= n[q]; p++) {
            double plane = (p - 0.5 * n[q]) * h[q];
            double a = (plane - S[q]) / dq;
            if (a > 0.0 && a < 1.0) buf[m++] = a;
        }
    }
    qsort(buf, (size_t)m, sizeof(double), og_cmp_double);
    return m;
}

/* flat index of the voxel containing point p, or -1 outside the grid */
static long og_voxel_at(const og_geom *g, const double p[3]) {
    int a = (int)floor(p[0] / g->hx + 0.5 * g->nx);
    int b = (int)floor(p[1] / g->hy + 0.5 * g->ny);
    int c = (int)floor(p[2] / g->hz + 0.5 * g->nz);
    if (a < 0 || a >= g->nx || b < 0 || b >= g->ny || c < 0 || c >= g->nz) return -1;
    return ((long)c * g->ny + b) * g->nx + a;
}

/* Siddon value of ray r (flat index view*nv*nu + j*nu + i); buf holds nx+ny+nz+8 doubles */
static double og_siddon_ray(const og_geom *g, const double *f, long r, double *buf) {
    int i = (int)(r % g->nu), j = (int)((r / g->nu) % g->nv), view = (int)(r / ((long)g->nu * g->nv));
    double S[3], D[3];
    og_ray_ends(g, view, i, j, S, D);
    double len = sqrt((D[0] - S[0]) * (D[0] - S[0]) + (D[1] - S[1]) * (D[1] - S[1]) + (D[2] - S[2]) * (D[2] - S[2]));
    int m = og_siddon_alphas(g, S, D, buf);
    double acc = 0.0;
    for (int k = 0; k + 1 < m; k++) {
        if (buf[k + 1] <= buf[k]) continue;
        double am = 0.5 * (buf[k] + buf[k + 1]), p[3];
        for (int q = 0; q < 3; q++) p[q] = S[q] + am * (D[q] - S[q]);
        long v = og_voxel_at(g, p);
        if (v >= 0) acc += (buf[k + 1] - buf[k]) * len * f[v];
    }
    return acc;
}

void orc_forward_siddon(const og_geom *g, const double *f, double *y) {
    long nray = og_nray(g);
    int cap = g->nx + g->ny + g->nz + 8;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
        for (long r = 0; r < nray; r++) y[r] = og_siddon_ray(g, f, r, buf);
        free(buf);
    }
}

/* Siddon P at selected rays */
void orc_forward_siddon_rays(const og_geom *g, const double *f, long n, const long *rays, double *out) {
    int cap = g->nx + g->ny + g->nz + 8;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)cap);
#pragma omp for schedule(dynamic, 16)
        for (long s = 0; s < n; s++) out[s] = og_siddon_ray(g, f, rays[s], buf);
        free(buf);
    }
}

/* Length of segment S -> D inside the box [lo, hi) (slab clipping; a segment running parallel to
 * a slab counts when its coordinate lies in [lo, hi)) */
static double og_box_chord(const double S[3], const double D[3], const double lo[3], const double hi[3]) {
    double t0 = 0.0, t1 = 1.0;
    for (int q = 0; q < 3; q++) {
        double d = D[q] - S[q];
        if (d == 0.0) {
            if (S[q] < lo[q] || S[q] >= hi[q]) return 0.0;
            continue;
        }
        double a = (lo[q] - S[q]) / d, b = (hi[q] - S[q]) / d;
        if (a > b) { double t = a; a = b; b = t; }
        if (a > t0) t0 = a;
        if (b < t1) t1 = b;
    }
    if (t1 <= t0) return 0.0;
    double len = sqrt((D[0] - S[0]) * (D[0] - S[0]) + (D[1] - S[1]) * (D[1] - S[1]) + (D[2] - S[2]) * (D[2] - S[2]));
    return (t1 - t0) * len;
}

/* (P_s^T y) at selected voxels: the sum over rays of (ray's length inside the voxel's cube) x y,
 * over the rays of each view whose pixel lies in the cube's projected bounding box */
void orc_adjoint_siddon_voxels(const og_geom *g, const double *y, long n, const long *vox, double *out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (long s = 0; s < n; s++) {
        long idx = vox[s];
        int a = (int)(idx % g->nx), b = (int)((idx / g->nx) % g->ny), c = (int)(idx / ((long)g->nx * g->ny));
        double lo[3] = {(a - 0.5 * g->nx) * g->hx, (b - 0.5 * g->ny) * g->hy, (c - 0.5 * g->nz) * g->hz};
        double hi[3] = {lo[0] + g->hx, lo[1] + g->hy, lo[2] + g->hz};
        double acc = 0.0;
        for (int view = 0; view < g->nviews; view++) {
            double th = og_angle(g, view);
            double ew[3] = {cos(th), sin(th), 0.0}, eu[3] = {sin(th), -cos(th), 0.0};
            double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
            for (int corner = 0; corner < 8; corner++) {
                double P[3] = {(corner & 1) ? hi[0] : lo[0], (corner & 2) ? hi[1] : lo[1], (corner & 4) ? hi[2] : lo[2]};
                double depth = (P[0] + g->sad * ew[0]) * ew[0] + (P[1] + g->sad * ew[1]) * ew[1];
                double uu = g->sdd * ((P[0] + g->sad * ew[0]) * eu[0] + (P[1] + g->sad * ew[1]) * eu[1]) / depth;
                double vv = g->sdd * P[2] / depth;
                if (uu < umin) umin = uu;
                if (uu > umax) umax = uu;
                if (vv < vmin) vmin = vv;
                if (vv > vmax) vmax = vv;
            }
            int i0 = (int)floor(umin / g->pu + 0.5 * (g->nu - 1)) - 1, i1 = (int)ceil(umax / g->pu + 0.5 * (g->nu - 1)) + 1;
            int j0 = (int)floor(vmin / g->pv + 0.5 * (g->nv - 1)) - 1, j1 = (int)ceil(vmax / g->pv + 0.5 * (g->nv - 1)) + 1;
            if (i0 < 0) i0 = 0;
            if (j0 < 0) j0 = 0;
            if (i1 > g->nu - 1) i1 = g->nu - 1;
            if (j1 > g->nv - 1) j1 = g->nv - 1;
            for (int j = j0; j <= j1; j++)
                for (int i = i0; i <= i1; i++) {
                    double S[3], D[3];
                    og_ray_ends(g, view, i, j, S, D);
                    acc += og_box_chord(S, D, lo, hi) * y[((long)view * g->nv + j) * g->nu + i];
                }
        }
        out[s] = acc;
    }
}

/* transpose of orc_forward_siddon (scatter into per-thread volumes, summed in thread order) */
void orc_adjoint_siddon(const og_geom *g, const double *y, double *f) {
    long nvox = og_nvox(g), nray = og_nray(g);
    int nt = orc_get_threads(), cap = g->nx + g->ny + g->nz + 8;
    double **vols = (double **)calloc((size_t)nt, sizeof(double *));
    for (int t = 0; t < nt; t++) vols[t] = (double *)calloc((size_t)nvox, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = vols[tid];
        double *buf = (double *)malloc(sizeof(double) * (size_t)cap);
#pragma omp for schedule(static)
        for (long r = 0; r < nray; r++) {
            if (y[r] == 0.0) continue;
            int i = (int)(r % g->nu), j = (int)((r / g->nu) % g->nv), view = (int)(r / ((long)g->nu * g->nv));
            double S[3], D[3];
            og_ray_ends(g, view, i, j, S, D);
            double len = sqrt((D[0] - S[0]) * (D[0] - S[0]) + (D[1] - S[1]) * (D[1] - S[1]) + (D[2] - S[2]) * (D[2] - S[2]));
            int m = og_siddon_alphas(g, S, D, buf);
            for (int k = 0; k + 1 < m; k++) {
                if (buf[k + 1] <= buf[k]) continue;
                double am = 0.5 * (buf[k] + buf[k + 1]), p[3];
                for (int q = 0; q < 3; q++) p[q] = S[q] + am * (D[q] - S[q]);
                long v = og_voxel_at(g, p);
                if (v >= 0) acc[v] += (buf[k + 1] - buf[k]) * len * y[r];
            }
        }
        free(buf);
    }
    for (long v = 0; v < nvox; v++) {
        double s = 0.0;
        for (int t = 0; t < nt; t++) s += vols[t][v];
        f[v] = s;
    }
    for (int t = 0; t < nt; t++) free(vols[t]);
    free(vols);
}

/* P at selected rays (flat indices view*nv*nu + j*nu + i) */
void orc_forward_rays(const og_geom *g, const double *f, long n, const long *rays, double *out) {
#pragma omp parallel for schedule(dynamic, 4)
    for (long s = 0; s < n; s++) {
        long r = rays[s];
        int i = (int)(r % g->nu);
        int j = (int)((r / g->nu) % g->nv);
        int view = (int)(r / ((long)g->nu * g->nv));
        out[s] = og_ray_integral(g, f, view, i, j);
    }
}

/* P^T by the transposed (scatter) loop; each thread scatters into its own volume and the
 * volumes are summed in thread order, so the result is reproducible for a thread count. */
void orc_adjoint(const og_geom *g, const double *y, double *f) {
    long nvox = og_nvox(g), nray = og_nray(g);
    int K = og_sample_halfwidth(g);
    int nt = orc_get_threads();
    double **buf = (double **)calloc((size_t)nt, sizeof(double *));
    for (int t = 0; t < nt; t++) buf[t] = (double *)calloc((size_t)nvox, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = buf[tid];
#pragma omp for schedule(static)
        for (long r = 0; r < nray; r++) {
            int i = (int)(r % g->nu);
            int j = (int)((r / g->nu) % g->nv);
            int view = (int)(r / ((long)g->nu * g->nv));
            og_ray ray;
            og_ray_setup(g, view, i, j, &ray);
            double val = ray.w * y[r], p[3];
            if (val == 0.0) continue;
            for (int k = -K; k <= K; k++) {
                og_sample_point(&ray, ray.tau_c + k * g->dtau, p);
                og_spread(g, acc, p, val);
            }
        }
    }
    for (long v = 0; v < nvox; v++) {
        double s = 0.0;
        for (int t = 0; t < nt; t++) s += buf[t][v];
        f[v] = s;
    }
    for (int t = 0; t < nt; t++) free(buf[t]);
    free(buf);
}

/* The voxel-driven backprojector of Section II.C.2 (Eq. 6, with the Jacobian of Eq. A7):
 * for every voxel centre V and view, the line from the source S through V meets the imager at
 * (u*, v*) (Eq. A6 rotated by theta); T is sampled there by bilinear interpolation between
 * pixel centres (zero beyond the imager) and weighted by L^3 / (L0 l^2), l = |V - S|,
 * L = |P - S|, L0 = SDD.  Scaled by hx hy hz / (pu pv), which makes it the continuum limit
 * of P^T (so it can stand in for P^T in Step 1 with the same step). */
static double og_bilinear_det(const og_geom *g, const double *T, int view, double u, double v) {
    double iu = u / g->pu + 0.5 * (g->nu - 1), iv = v / g->pv + 0.5 * (g->nv - 1);
    int i0 = (int)floor(iu), j0 = (int)floor(iv);
    double s = 0.0;
    for (int j = j0; j <= j0 + 1; j++) {
        if (j < 0 || j >= g->nv) continue;
        for (int i = i0; i <= i0 + 1; i++) {
            if (i < 0 || i >= g->nu) continue;
            s += T[((long)view * g->nv + j) * g->nu + i] * og_hat(iu - i) * og_hat(iv - j);
        }
    }
    return s;
}

void orc_backproject_eq6(const og_geom *g, const double *T, double *f) {
    const double scale = g->hx * g->hy * g->hz / (g->pu * g->pv);
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < og_nvox(g); idx++) {
        int a = (int)(idx % g->nx), b = (int)((idx / g->nx) % g->ny), c = (int)(idx / ((long)g->nx * g->ny));
        double V[3] = {(a - 0.5 * (g->nx - 1)) * g->hx, (b - 0.5 * (g->ny - 1)) * g->hy,
                       (c - 0.5 * (g->nz - 1)) * g->hz};
        double acc = 0.0;
        for (int view = 0; view < g->nviews; view++) {
            double th = og_angle(g, view);
            double ew[3] = {cos(th), sin(th), 0.0}, eu[3] = {sin(th), -cos(th), 0.0};
            double S[3] = {-g->sad * ew[0], -g->sad * ew[1], 0.0};
            double d[3] = {V[0] - S[0], V[1] - S[1], V[2] - S[2]};
            double depth = d[0] * ew[0] + d[1] * ew[1];       /* along the central ray */
            double us = g->sdd * (d[0] * eu[0] + d[1] * eu[1]) / depth;
            double vs = g->sdd * d[2] / depth;
            double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double L = sqrt(g->sdd * g->sdd + us * us + vs * vs);
            const double jac = (og_fault == 12) ? L * L : L * L * L;
            acc += jac / (g->sdd * l * l) * og_bilinear_det(g, T, view, us, vs);
        }
        f[idx] = scale * acc;
    }
}

/* P^T at selected voxels (flat indices (c*ny + b)*nx + a).  Only rays whose pixel lies in
 * the detector footprint of the voxel's support (its centre +- one voxel) can reach it;
 * the sum runs over those rays and all their samples. */
void orc_adjoint_voxels(const og_geom *g, const double *y, long n, const long *vox, double *out) {
    int K = og_sample_halfwidth(g);
#pragma omp parallel for schedule(dynamic, 1)
    for (long s = 0; s < n; s++) {
        long idx = vox[s];
        int a = (int)(idx % g->nx), b = (int)((idx / g->nx) % g->ny), c = (int)(idx / ((long)g->nx * g->ny));
        double xc[3] = {(a - 0.5 * (g->nx - 1)) * g->hx, (b - 0.5 * (g->ny - 1)) * g->hy,
                        (c - 0.5 * (g->nz - 1)) * g->hz};
        double acc = 0.0;
        for (int view = 0; view < g->nviews; view++) {
            double th = og_angle(g, view);
            double ew[3] = {cos(th), sin(th), 0.0}, eu[3] = {sin(th), -cos(th), 0.0};
            double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
            for (int corner = 0; corner < 8; corner++) {
                double P[3] = {xc[0] + ((corner & 1) ? g->hx : -g->hx), xc[1] + ((corner & 2) ? g->hy : -g->hy),
                               xc[2] + ((corner & 4) ? g->hz : -g->hz)};
                double rel[3] = {P[0] + g->sad * ew[0], P[1] + g->sad * ew[1], P[2]};
                double depth = rel[0] * ew[0] + rel[1] * ew[1];
                double uu = g->sdd * (rel[0] * eu[0] + rel[1] * eu[1]) / depth;
                double vv = g->sdd * rel[2] / depth;
                if (uu < umin) umin = uu;
                if (uu > umax) umax = uu;
                if (vv < vmin) vmin = vv;
                if (vv > vmax) vmax = vv;
            }
            int i0 = (int)floor(umin / g->pu + 0.5 * (g->nu - 1)) - 1, i1 = (int)ceil(umax / g->pu + 0.5 * (g->nu - 1)) + 1;
            int j0 = (int)floor(vmin / g->pv + 0.5 * (g->nv - 1)) - 1, j1 = (int)ceil(vmax / g->pv + 0.5 * (g->nv - 1)) + 1;
            if (og_fault == 14) { i0 += 3; i1 -= 3; j0 += 3; j1 -= 3; }
            if (i0 < 0) i0 = 0;
            if (j0 < 0) j0 = 0;
            if (i1 > g->nu - 1) i1 = g->nu - 1;
            if (j1 > g->nv - 1) j1 = g->nv - 1;
            for (int j = j0; j <= j1; j++)
                for (int i = i0; i <= i1; i++) {
                    og_ray ray;
                    og_ray_setup(g, view, i, j, &ray);
                    double val = ray.w * y[((long)view * g->nv + j) * g->nu + i], p[3], q[3];
                    if (val == 0.0) continue;
                    for (int k = -K; k <= K; k++) {
                        og_sample_point(&ray, ray.tau_c + k * g->dtau, p);
                        og_index_coords(g, p, q);
                        acc += val * og_hat(q[0] - a) * og_hat(q[1] - b) * og_hat(q[2] - c);
                    }
                }
        }
        out[s] = acc;
    }
}

/* ---------------------------------------------------------------------------------- */
/* Total variation (E1 of Eq. 2, smoothed; boundary conditions of Section II.B)        */
/* ---------------------------------------------------------------------------------- */
#define OG_F(f, a, b, c) (f)[((long)(c) * g->ny + (b)) * g->nx + (a)]

static void og_diffs(const og_geom *g, const double *f, int a, int b, int c, double D[3]) {
    double f0 = OG_F(f, a, b, c);
    double fx = (a + 1 < g->nx) ? OG_F(f, a + 1, b, c) : 0.0; /* zero BC (lateral) */
    double fy = (b + 1 < g->ny) ? OG_F(f, a, b + 1, c) : 0.0; /* zero BC (AP) */
    double fz = (c + 1 < g->nz) ? OG_F(f, a, b, c + 1) : (og_fault == 5 ? 0.0 : f0); /* reflective (SI) */
    D[0] = (fx - f0) / g->hx;
    D[1] = (fy - f0) / g->hy;
    D[2] = (fz - f0) / g->hz;
}

/* R(f) = mean over voxels of sqrt(|D f|^2 + eps^2) */
double orc_tv_energy(const og_geom *g, const double *f, double eps) {
    double s = 0.0;
    for (int c = 0; c < g->nz; c++)
        for (int b = 0; b < g->ny; b++)
            for (int a = 0; a < g->nx; a++) {
                double D[3];
                og_diffs(g, f, a, b, c, D);
                s += sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2] + eps * eps);
            }
    return s / (double)og_nvox(g);
}

/* dR/df (chain rule through every forward difference, as a scatter loop) */
void orc_tv_grad(const og_geom *g, const double *f, double eps, double *grad) {
    long nvox = og_nvox(g);
    double inv_n = 1.0 / (double)nvox;
    memset(grad, 0, sizeof(double) * (size_t)nvox);
    for (int c = 0; c < g->nz; c++)
        for (int b = 0; b < g->ny; b++)
            for (int a = 0; a < g->nx; a++) {
                double D[3];
                og_diffs(g, f, a, b, c, D);
                double phi = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2] + eps * eps);
                double qx = D[0] / phi * inv_n, qy = D[1] / phi * inv_n, qz = D[2] / phi * inv_n;
                /* D_x = (f_{a+1} - f_a)/hx: f_a always enters (the ghost is a constant 0) */
                OG_F(grad, a, b, c) -= qx / g->hx;
                if (a + 1 < g->nx) OG_F(grad, a + 1, b, c) += qx / g->hx;
                if (og_fault != 6) {
                    OG_F(grad, a, b, c) -= qy / g->hy;
                    if (b + 1 < g->ny) OG_F(grad, a, b + 1, c) += qy / g->hy;
                }
                /* D_z at the last plane is identically 0 (reflective ghost) */
                if (c + 1 < g->nz) {
                    OG_F(grad, a, b, c) -= qz / g->hz;
                    OG_F(grad, a, b, c + 1) += qz / g->hz;
                } else if (og_fault == 5) {
                    OG_F(grad, a, b, c) -= qz / g->hz;
                }
            }
}

/* ---------------------------------------------------------------------------------- */
/* Step 2: ROF sub-problem by gradient descent with the Armijo rule (Eq. 5)           */
/* ---------------------------------------------------------------------------------- */
/* E_R(u) = lambda R(u) + (1/(2t)) mean((u-g)^2) */
static double og_rof_energy(const og_geom *g, const double *u, const double *gg, const og_params *pr,
                            double t) {
    long n = og_nvox(g);
    double q = 0.0;
    for (long v = 0; v < n; v++) q += (u[v] - gg[v]) * (u[v] - gg[v]);
    return pr->lambda * orc_tv_energy(g, u, pr->tv_eps) + q / (double)n / (2.0 * t);
}

typedef struct {
    og_stats *st;
    int level, outer;
} og_trace_ctx;

static void og_record(og_trace_ctx *tc, int inner, int m, double e0, double e1, double G) {
    if (!tc || !tc->st) return;
    og_stats *st = tc->st;
    int k = st->trace_len;
    if (st->trace && k < st->trace_cap) {
        st->trace[4 * k + 0] = tc->level;
        st->trace[4 * k + 1] = tc->outer;
        st->trace[4 * k + 2] = inner;
        st->trace[4 * k + 3] = m;
        if (st->rof_e) {
            st->rof_e[3 * k + 0] = e0;
            st->rof_e[3 * k + 1] = e1;
            st->rof_e[3 * k + 2] = G;
        }
    }
    st->trace_len = k + 1;
}

/* u = argmin approx of lambda R(u) + (1/(2t)) mean((u-g)^2), from u = g.  The search
 * direction d is the gradient with respect to the normalised measure dV/V, i.e. N times
 * the plain derivative; the Armijo test uses G = mean(d^2) for (1/V) int d^2. */
static void og_rof(const og_geom *g, const double *gg, double *u, const og_params *pr, double t,
                   og_trace_ctx *tc) {
    long n = og_nvox(g);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    double *trial = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(u, gg, sizeof(double) * (size_t)n);
    for (int it = 0; it < pr->rof_max_iter; it++) {
        double e0 = og_rof_energy(g, u, gg, pr, t);
        orc_tv_grad(g, u, pr->tv_eps, d);
        double G = 0.0;
        for (long v = 0; v < n; v++) {
            d[v] = pr->lambda * (double)n * d[v] + (u[v] - gg[v]) / t;
            G += d[v] * d[v];
        }
        G /= (double)n;
        double s = t, enew = 0.0;
        int m = 0, ok = 0;
        for (;;) {
            for (long v = 0; v < n; v++) trial[v] = u[v] - s * d[v];
            enew = og_rof_energy(g, trial, gg, pr, t);
            double bound = e0 - pr->armijo_c * s * G;
            if (og_fault == 8) bound = e0 + pr->armijo_c * s * G;
            if (enew <= bound) { ok = 1; break; }
            if (m >= pr->rof_max_backtrack) break;
            s *= pr->backtrack;
            m++;
        }
        og_record(tc, it, ok ? m : -1, e0, enew, G);
        if (!ok) break; /* no step satisfied Eq. 5: keep u */
        memcpy(u, trial, sizeof(double) * (size_t)n);
        if (og_fault == 15) continue;
        if (e0 == 0.0 || G == 0.0 || fabs(enew - e0) / e0 < pr->rof_tol) break;
    }
    free(d);
    free(trial);
}

/* ---------------------------------------------------------------------------------- */
/* Algorithm A1 on one grid                                                           */
/* ---------------------------------------------------------------------------------- */
/* the operator pair of the reconstruction */
static void og_P(const og_geom *g, int projector, const double *f, double *y) {
    if (projector == 1) orc_forward_siddon(g, f, y);
    else orc_forward(g, f, y);
}
static void og_PT(const og_geom *g, int projector, const double *y, double *f) {
    if (projector == 1) orc_adjoint_siddon(g, y, f);
    else orc_adjoint(g, y, f);
}

static double og_data_term(const og_geom *g, int projector, const double *f, const double *Y, double *r) {
    long nr = og_nray(g);
    og_P(g, projector, f, r);
    double s = 0.0;
    for (long q = 0; q < nr; q++) {
        r[q] -= Y[q];
        s += r[q] * r[q];
    }
    return s / (double)nr;
}

/* max(P 1) and max(P^T 1): the Schur bound ||P||_2^2 <= max row sum * max column sum */
static void og_schur(const og_geom *g, int projector, double *max_p1, double *max_pt1) {
    long nvox = og_nvox(g), nr = og_nray(g);
    double *one_v = (double *)malloc(sizeof(double) * (size_t)nvox);
    double *one_r = (double *)malloc(sizeof(double) * (size_t)nr);
    double *tv = (double *)malloc(sizeof(double) * (size_t)nvox);
    double *tr = (double *)malloc(sizeof(double) * (size_t)nr);
    for (long v = 0; v < nvox; v++) one_v[v] = 1.0;
    for (long q = 0; q < nr; q++) one_r[q] = 1.0;
    og_P(g, projector, one_v, tr);
    og_PT(g, projector, one_r, tv);
    double m1 = 0.0, m2 = 0.0;
    for (long q = 0; q < nr; q++) if (tr[q] > m1) m1 = tr[q];
    for (long v = 0; v < nvox; v++) if (tv[v] > m2) m2 = tv[v];
    *max_p1 = m1;
    *max_pt1 = m2;
    free(one_v); free(one_r); free(tv); free(tr);
}

void orc_schur(const og_geom *g, double *max_p1, double *max_pt1) { og_schur(g, 0, max_p1, max_pt1); }

/* step scale of Step 1: g = f - t * kappa0 * P^T r, kappa0 = 2 N_vox / (N_theta N_pix) */
static double og_kappa0(const og_geom *g) { return 2.0 * (double)og_nvox(g) / (double)og_nray(g); }

static double og_schur_step(const og_geom *g, int projector) {
    double a, b;
    og_schur(g, projector, &a, &b);
    return 1.0 / ((og_fault == 18 ? 0.5 : 1.0) * og_kappa0(g) * a * b);
}

double orc_schur_step(const og_geom *g) { return og_schur_step(g, 0); }

static void og_energy_push(og_stats *st, double e) {
    if (!st) return;
    if (st->energy && st->energy_len < st->energy_cap) st->energy[st->energy_len] = e;
    st->energy_len++;
}

/* `iters` outer iterations of Algorithm A1 from f (in/out) */
void orc_fbs(const og_geom *g, const double *Y, double *f, int iters, const og_params *pr, double t,
             og_stats *st, int level) {
    long nvox = og_nvox(g), nr = og_nray(g);
    double *r = (double *)malloc(sizeof(double) * (size_t)nr);
    double *pt = (double *)malloc(sizeof(double) * (size_t)nvox);
    double *gg = (double *)malloc(sizeof(double) * (size_t)nvox);
    double *u = (double *)malloc(sizeof(double) * (size_t)nvox);
    double kappa = t * og_kappa0(g) * (og_fault == 16 ? 0.5 : 1.0);
    og_trace_ctx tc = {st, level, 0};
    double e_prev = 0.0;
    int converged = 0;
    for (int k = 0; k < iters; k++) {
        /* Step 1: gradient step on the data term, g = f - t N dD/df */
        double Dk = og_data_term(g, pr->projector, f, Y, r);
        double Ek = Dk + pr->lambda * orc_tv_energy(g, f, pr->tv_eps);
        og_energy_push(st, Ek);
        /* "until convergence" (Section II.C.3): f_k is final once the energy stalls */
        if (pr->conv_tol > 0.0 && k >= 1 && fabs(Ek - e_prev) <= pr->conv_tol * e_prev) {
            converged = 1;
            break;
        }
        e_prev = Ek;
        if (pr->step1_eq6) orc_backproject_eq6(g, r, pt);
        else og_PT(g, pr->projector, r, pt);
        for (long v = 0; v < nvox; v++) gg[v] = (og_fault == 9) ? f[v] + kappa * pt[v] : f[v] - kappa * pt[v];
        /* Step 2: ROF */
        tc.outer = k;
        og_rof(g, gg, u, pr, t, &tc);
        /* Step 3: non-negativity */
        for (long v = 0; v < nvox; v++) f[v] = u[v] > 0.0 ? u[v] : 0.0;
    }
    if (st && !converged) {
        double Dk = og_data_term(g, pr->projector, f, Y, r);
        og_energy_push(st, Dk + pr->lambda * orc_tv_energy(g, f, pr->tv_eps));
    }
    free(r); free(pt); free(gg); free(u);
}

/* ---------------------------------------------------------------------------------- */
/* Multigrid transfers (Section II.C.3)                                               */
/* ---------------------------------------------------------------------------------- */
/* weight of coarse sample cc (of n) in fine sample F (of 2n): 3/4 parent, 1/4 the
 * coarse neighbour on F's side, indices clamped (a clamped neighbour adds to the parent) */
static double og_prol_w(int F, int cc, int n) {
    int parent = F / 2;
    int nb = (F % 2 == 0) ? parent - 1 : parent + 1;
    if (nb < 0) nb = 0;
    if (nb > n - 1) nb = n - 1;
    double wp = (og_fault == 7) ? 0.5 : 0.75, wn = (og_fault == 7) ? 0.5 : 0.25;
    double w = 0.0;
    if (cc == parent) w += wp;
    if (cc == nb) w += wn;
    return w;
}

/* fine (2nx, 2ny, 2nz) from coarse (nx, ny, nz) */
void orc_prolong(int nx, int ny, int nz, const double *coarse, double *fine) {
    int NX = 2 * nx, NY = 2 * ny, NZ = 2 * nz;
    for (int C = 0; C < NZ; C++)
        for (int B = 0; B < NY; B++)
            for (int A = 0; A < NX; A++) {
                double s = 0.0;
                for (int c = (C / 2) - 1; c <= (C / 2) + 1; c++) {
                    if (c < 0 || c >= nz) continue;
                    double wz = og_prol_w(C, c, nz);
                    for (int b = (B / 2) - 1; b <= (B / 2) + 1; b++) {
                        if (b < 0 || b >= ny) continue;
                        double wy = og_prol_w(B, b, ny);
                        for (int a = (A / 2) - 1; a <= (A / 2) + 1; a++) {
                            if (a < 0 || a >= nx) continue;
                            s += og_prol_w(A, a, nx) * wy * wz * coarse[((long)c * ny + b) * nx + a];
                        }
                    }
                }
                fine[((long)C * NY + B) * NX + A] = s;
            }
}

/* coarse = (1/8) Prol^T fine, as the transposed scatter */
void orc_restrict(int nx, int ny, int nz, const double *fine, double *coarse) {
    int NX = 2 * nx, NY = 2 * ny, NZ = 2 * nz;
    double scale = (og_fault == 10) ? 1.0 : 0.125;
    memset(coarse, 0, sizeof(double) * (size_t)nx * ny * nz);
    for (int C = 0; C < NZ; C++)
        for (int B = 0; B < NY; B++)
            for (int A = 0; A < NX; A++) {
                double val = fine[((long)C * NY + B) * NX + A];
                for (int c = (C / 2) - 1; c <= (C / 2) + 1; c++) {
                    if (c < 0 || c >= nz) continue;
                    double wz = og_prol_w(C, c, nz);
                    for (int b = (B / 2) - 1; b <= (B / 2) + 1; b++) {
                        if (b < 0 || b >= ny) continue;
                        double wy = og_prol_w(B, b, ny);
                        for (int a = (A / 2) - 1; a <= (A / 2) + 1; a++) {
                            if (a < 0 || a >= nx) continue;
                            coarse[((long)c * ny + b) * nx + a] += scale * og_prol_w(A, a, nx) * wy * wz * val;
                        }
                    }
                }
            }
}

/* detector restriction: mean over f x f pixel blocks */
void orc_bin_detector(int nviews, int nv, int nu, int factor, const double *Y, double *out) {
    int mv = nv / factor, mu = nu / factor;
    for (int view = 0; view < nviews; view++)
        for (int j = 0; j < mv; j++)
            for (int i = 0; i < mu; i++) {
                double s = 0.0;
                for (int jj = 0; jj < factor; jj++)
                    for (int ii = 0; ii < factor; ii++)
                        s += Y[((long)view * nv + j * factor + jj) * nu + i * factor + ii];
                out[((long)view * mv + j) * mu + i] = s / (double)(factor * factor);
            }
}

/* geometry of multigrid level l: grid halved l times over the same box; detector binned
 * when bin_detector; sample spacing scales with the grid */
void orc_level_geom(const og_geom *g0, int l, int bin_detector, og_geom *gl) {
    int f = 1 << l;
    *gl = *g0;
    gl->nx = g0->nx / f; gl->ny = g0->ny / f; gl->nz = g0->nz / f;
    gl->hx = g0->hx * f; gl->hy = g0->hy * f; gl->hz = g0->hz * f;
    if (bin_detector) {
        gl->nu = g0->nu / f; gl->nv = g0->nv / f;
        gl->pu = g0->pu * (og_fault == 17 ? 1 : f); gl->pv = g0->pv * (og_fault == 17 ? 1 : f);
    }
    gl->dtau = g0->dtau * (og_fault == 19 ? 1 : f);
}

/* P of multigrid level l (orc_level_geom of g0) applied to a level-l volume */
void orc_forward_level(const og_geom *g0, int l, int bin_detector, const double *f, double *y) {
    og_geom gl;
    orc_level_geom(g0, l, bin_detector, &gl);
    orc_forward(&gl, f, y);
}

/* Full reconstruction: levels from the coarsest (levels-1) to the finest (0), each started
 * from the prolonged solution of the next coarser level (f = 0, or the restricted d_init,
 * on the coarsest).  Returns 0, or -1 when the grid is not divisible by 2^(levels-1). */
int orc_reconstruct(const og_geom *g0, int levels, const int *iters, const og_params *pr, int bin_detector,
                    const double *Y0, const double *d_init, double *f_out, og_stats *st) {
    int fct = 1 << (levels - 1);
    if (levels < 1 || levels > 16) return -1;
    if (g0->nx % fct || g0->ny % fct || g0->nz % fct) return -1;
    if (bin_detector && (g0->nu % fct || g0->nv % fct)) return -1;
    if (st) { st->trace_len = 0; st->energy_len = 0; }
    double *f = NULL;
    og_geom gl;
    /* coarsest start */
    orc_level_geom(g0, levels - 1, bin_detector, &gl);
    f = (double *)calloc((size_t)og_nvox(&gl), sizeof(double));
    if (d_init) {
        double *cur = (double *)malloc(sizeof(double) * (size_t)og_nvox(g0));
        memcpy(cur, d_init, sizeof(double) * (size_t)og_nvox(g0));
        for (int l = 1; l < levels; l++) {
            og_geom gc;
            orc_level_geom(g0, l, bin_detector, &gc);
            double *nxt = (double *)malloc(sizeof(double) * (size_t)og_nvox(&gc));
            orc_restrict(gc.nx, gc.ny, gc.nz, cur, nxt);
            free(cur);
            cur = nxt;
        }
        memcpy(f, cur, sizeof(double) * (size_t)og_nvox(&gl));
        free(cur);
    }
    for (int l = levels - 1; l >= 0; l--) {
        orc_level_geom(g0, l, bin_detector, &gl);
        if (l < levels - 1) {
            double *fine = (double *)malloc(sizeof(double) * (size_t)og_nvox(&gl));
            orc_prolong(gl.nx / 2, gl.ny / 2, gl.nz / 2, f, fine);
            free(f);
            f = fine;
        }
        double *Yl;
        if (bin_detector && l > 0) {
            Yl = (double *)malloc(sizeof(double) * (size_t)og_nray(&gl));
            orc_bin_detector(g0->nviews, g0->nv, g0->nu, 1 << l, Y0, Yl);
        } else {
            Yl = (double *)Y0;
        }
        double t = pr->step > 0.0 ? pr->step : og_schur_step(&gl, pr->projector);
        if (st && l < 16) st->t_used[l] = t;
        orc_fbs(&gl, Yl, f, iters[l], pr, t, st, l);
        if (Yl != Y0) free(Yl);
    }
    memcpy(f_out, f, sizeof(double) * (size_t)og_nvox(g0));
    free(f);
    return 0;
}

/* ROF alone (Step 2) on one grid, for unit tests of the inner solver */
void orc_rof(const og_geom *g, const double *gg, double *u, const og_params *pr, double t, og_stats *st) {
    og_trace_ctx tc = {st, 0, 0};
    if (st) st->trace_len = 0;
    og_rof(g, gg, u, pr, t, &tc);
}
