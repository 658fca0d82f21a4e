/*
 * libcbct — TV-regularised cone-beam CT reconstruction on AMD Instinct MI355X (gfx950).
 *
 * The calls follow the problem statement of Jia et al., "GPU-based fast low-dose cone beam
 * CT reconstruction via total variation": a circular cone-beam geometry (Section II.A, Eq. 1,
 * Fig. 1; Section III.A for SAD/SDD), projections Y (Eq. 1-2), a regularisation weight
 * (Eq. 2, here lambda = 1/mu on the TV term), outer iterations of Algorithm A1 (Section II.B)
 * and multigrid levels (Section II.C.3).
 *
 * Conventions shared by every call
 *   Coordinates  x lateral, y anterior-posterior, z superior-inferior (rotation axis), mm.
 *                Voxel centres x_a = (a - (nx-1)/2) hx (same for y, z): the grid is centred
 *                on the isocentre.  View theta: source S = -sad (cos t, sin t, 0); detector
 *                pixel (i, j) at S + sdd e_w + u_i e_u + v_j e_z with e_w = (cos t, sin t, 0),
 *                e_u = (sin t, -cos t, 0), u_i = (i - (nu-1)/2) pu, v_j = (j - (nv-1)/2) pv.
 *                (At theta = 0 this is the geometry of Appendix Eqs. A2 and A6.)
 *   Layouts      volume  float32 [nz][ny][nx] (x fastest), C-contiguous;
 *                projections float32 [n_views][nv][nu] (u fastest), C-contiguous.
 *   P            (P f)_{t,j,i} = w_ij * sum_k f~(p_k): the ray integral of Eq. 1 through the
 *                zero-extended trilinear interpolant f~ of the voxel grid, sampled where the
 *                ray's transverse distance from S is tau_c,i + k*dtau (tau_c,i: closest
 *                approach of detector column i's transverse line to the axis; dtau =
 *                sample_ratio * min(hx, hy) at level 0).  w_ij = dtau * |D_ij - S| / |D_ij - S|_xy.
 *   P^T          the exact transpose of P (Section II.C.2: the data-term gradient is
 *                P^T (P f - Y) up to constants), computed by a voxel-driven gather.
 *   Devices      a context names the HIP device the library works on (the paper's single
 *                GPU); plans and servers are created from a context and keep its device:
 *                every call on a plan runs with that device current and restores the
 *                caller's device before it returns.
 *   Memory       every d_* pointer is device memory on the plan's device, owned by the caller.
 *                The library owns only contexts, plans (geometry tables) and servers.  No call
 *                allocates device memory except cbct_plan_create and the server calls.
 *   Streams      every call is asynchronous on `stream` (0 = the null stream) unless stated.
 *   Errors       the status code is the only error channel; nothing aborts or throws across
 *                the ABI.  On error, cbct_last_error() (thread-local) describes it.
 *                CBCT_ERR_INVALID_ARG is returned before any work is queued.
 *   Threads      plans are immutable after creation and may be used from several threads
 *                and streams at once, as long as each call gets its own workspace.
 */
#ifndef CBCT_H
#define CBCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *cbct_stream_t; /* a hipStream_t */

typedef enum {
    CBCT_OK = 0,
    CBCT_ERR_INVALID_ARG = 1,   /* bad pointer, size, geometry, level or workspace */
    CBCT_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed */
    CBCT_ERR_BUDGET = 3,        /* a request does not fit the server's HBM budget */
    CBCT_ERR_HIP = 4,           /* a HIP runtime call failed (message has the HIP error) */
    CBCT_ERR_NONFINITE = 5,     /* a reduction produced NaN or Inf */
    CBCT_ERR_NOT_FOUND = 6,     /* unknown server ticket */
    CBCT_ERR_INTERNAL = 7
} cbct_status;

/* Scan geometry (Section II.A, Fig. 1).  Lengths in mm, angles in radians. */
typedef struct {
    int nx, ny, nz;        /* voxels */
    double hx, hy, hz;     /* voxel pitch */
    int nu, nv;            /* detector columns (u) and rows (v) */
    double pu, pv;         /* detector pitch */
    double sad, sdd;       /* source-axis and source-detector distances (L0 of the paper) */
    int n_views;
    const double *angles;  /* n_views angles, or NULL for 2*pi*k/n_views; copied at plan creation */
    double sample_ratio;   /* rho: dtau = rho * min(hx, hy); <= 0 means 1 */
} cbct_geometry_desc;

typedef struct cbct_context cbct_context;
typedef struct cbct_plan cbct_plan;

/* The device the reconstruction runs on (the paper runs Algorithm A1 on one GPU, Section
 * II.C): checks that HIP device `hip_device` exists and is a gfx950 (the only code objects the
 * library carries) and returns a handle that plans and servers are created from.  The caller
 * owns it and destroys it after every plan and server made from it (a server keeps a copy of
 * the device, so it may outlive the context).  Errors: INVALID_ARG for a NULL out, a device
 * outside [0, device count) or another architecture; HIP; OUT_OF_MEMORY.  No device memory is
 * allocated. */
cbct_status cbct_context_create(int hip_device, cbct_context **out);
void cbct_context_destroy(cbct_context *ctx);
/* the context's HIP device ordinal */
cbct_status cbct_context_device(const cbct_context *ctx, int *hip_device);

/* Builds the geometry tables for `levels` multigrid levels (Section II.C.3) on the context's
 * device.  Level l has dims n/2^l over the same box (pitch h*2^l), sample spacing dtau*2^l and,
 * when bin_detector != 0, a detector binned 2^l x 2^l (pitch p*2^l).
 * Errors: INVALID_ARG for a NULL context, non-positive sizes, sad <= half the grid diagonal,
 * sdd <= sad, or dims (and detector dims when binning) not divisible by 2^(levels-1);
 * OUT_OF_MEMORY; HIP. */
cbct_status cbct_plan_create(cbct_context *ctx, const cbct_geometry_desc *geom, int levels, int bin_detector,
                             cbct_plan **out);
void cbct_plan_destroy(cbct_plan *plan);

/* dims of a level: out[0..4] = nx, ny, nz, nu, nv; out[5] = n_views */
cbct_status cbct_plan_level_dims(const cbct_plan *plan, int level, int out[6]);

/* Workspace (device bytes) that cbct_forward needs at `level`: one volume in the kernels'
 * column-major layout.  The caller allocates it; calls running at once need separate ones. */
cbct_status cbct_forward_workspace_size(const cbct_plan *plan, int level, size_t *bytes);

/* Forward projection P (Eq. 1): d_proj = P_level d_vol.
 * d_vol [nz][ny][nx] and d_proj [n_views][nv][nu] at the level's dims; d_ws of at least
 * cbct_forward_workspace_size bytes.  INVALID_ARG on NULL pointers, a bad level or a small
 * workspace. */
cbct_status cbct_forward(const cbct_plan *plan, int level, const float *d_vol, float *d_proj, void *d_ws,
                         size_t ws_bytes, cbct_stream_t stream);

/* The same P for a volume already in the projector's column-major layout [ny][nx][nz]
 * (z fastest), as the reconstruction keeps it: no workspace, one kernel. */
cbct_status cbct_forward_columns(const cbct_plan *plan, int level, const float *d_vol_cols, float *d_proj,
                                 cbct_stream_t stream);

/* The paper's voxel-driven backprojector (Section II.C.2, Eq. 6 with the Jacobian of Eq. A7):
 * d_vol = B_level d_proj, where for every voxel centre V and view the line from the source
 * through V meets the imager at (u*, v*) (Eq. A6), d_proj is sampled there by bilinear
 * interpolation between pixel centres (zero beyond the imager) and weighted by L^3 / (L0 l^2);
 * the sum over views is scaled by hx hy hz / (pu pv) (the continuum limit of P^T, not its exact
 * transpose).  d_proj [n_views][nv][nu], d_vol [nz][ny][nx] at `level`, device memory.  No
 * workspace, no atomics.  Errors: CBCT_ERR_INVALID_ARG for a NULL pointer or a bad level. */
cbct_status cbct_backproject_eq6(const cbct_plan *plan, int level, const float *d_proj, float *d_vol,
                                 cbct_stream_t stream);

/* Siddon's exact radiological path (the ray tracer of Section II.C.2 and the data simulator of
 * Section III.A) as an alternative projector: each voxel is constant on its cube (half-open on the
 * upper faces) and d_proj = P_s d_vol holds, per ray S -> D, the sum over voxels of the length of
 * S -> D inside the cube times the voxel value.  d_vol [nz][ny][nx], d_proj [n_views][nv][nu] at
 * `level`, device memory; d_ws of at least cbct_forward_workspace_size bytes (the same column-major
 * copy of the volume as cbct_forward).  INVALID_ARG on NULL pointers, a bad level or a small
 * workspace. */
cbct_status cbct_forward_siddon(const cbct_plan *plan, int level, const float *d_vol, float *d_proj, void *d_ws,
                                size_t ws_bytes, cbct_stream_t stream);

/* Workspace (device bytes) of cbct_adjoint_siddon at `level`: a z profile (nz floats) for every
 * piece of every detector column's transverse line (n_views x nu x (nx + ny + 3) x nz floats) plus
 * 16 bytes per column. */
cbct_status cbct_adjoint_siddon_workspace_size(const cbct_plan *plan, int level, size_t *bytes);

/* Transpose of cbct_forward_siddon: d_vol = P_s^T d_proj (the matched backprojector; Section
 * II.C.2 explains why it is voxel-driven): each voxel gathers length x value over the rays that
 * cross its cube.  d_proj [n_views][nv][nu], d_vol [nz][ny][nx] at `level`; d_ws: at least
 * cbct_adjoint_siddon_workspace_size bytes, 256-byte aligned, overwritten.  Every voxel of d_vol is
 * written once, no atomics.  INVALID_ARG on NULL pointers, a bad level or a small or misaligned
 * workspace. */
cbct_status cbct_adjoint_siddon(const cbct_plan *plan, int level, const float *d_proj, float *d_vol, void *d_ws,
                                size_t ws_bytes, cbct_stream_t stream);

/* Workspace (device bytes) of cbct_adjoint at `level`: the z profiles of every detector
 * column's samples (views x columns x samples in the grid's support x nz floats). */
cbct_status cbct_adjoint_workspace_size(const cbct_plan *plan, int level, size_t *bytes);

/* Adjoint P^T (exact transpose of cbct_forward; Section II.C.2): d_vol = P_level^T d_proj.
 * d_ws: >= cbct_adjoint_workspace_size bytes, 16-byte aligned.  The voxel-driven gather writes
 * every voxel of d_vol once and uses no atomics. */
cbct_status cbct_adjoint(const cbct_plan *plan, int level, const float *d_proj, float *d_vol, void *d_ws,
                         size_t ws_bytes, cbct_stream_t stream);

/* ---- Reconstruction: Algorithm A1 (Section II.B) with the multigrid cascade (II.C.3) ------
 *
 * Energy (Eq. 2 in lambda form, 1/V and 1/(N_theta A) read as means):
 *   E(f) = mean((P f - Y)^2) + lambda mean(sqrt(|D f|^2 + tv_eps^2)),  f >= 0,
 * D = forward differences with ghost 0 beyond the last x and y sample and ghost = last plane
 * beyond the last z plane (boundary conditions of Section II.B).  Each outer iteration:
 *   Step 1  g = f - t kappa0 P^T (P f - Y),  kappa0 = 2 N_vox / (n_views nu nv)
 *   Step 2  u = g, then ROF gradient descent on E_R(u) = lambda R(u) + mean((u-g)^2)/(2t) along
 *           d = lambda N dR/du + (u-g)/t: step s = t alpha^m with the least m <= rof_max_backtrack
 *           such that E_R(u - s d) <= E_R(u) - armijo_c s mean(d^2) (Eq. 5); no such m: stop;
 *           stop also when |E_new - E_0| / E_0 < rof_tol or after rof_max_iter iterations
 *   Step 3  f = max(u, 0)
 * Levels run from params.levels-1 (coarsest, started from 0 or from d_init restricted) to 0,
 * each started from the prolonged solution of the coarser one; t = params.step, or when
 * step <= 0 the Schur bound 1 / (kappa0 max(P_l 1) max(P_l^T 1)) per level (cached in the plan).
 * params.projector picks the pair P, P^T: the trilinear sampling pair (the line integral of
 * Eq. 1 and its exact adjoint) or the Siddon pair of exact ray-in-voxel lengths (the ray tracer
 * of Section II.C.2), everywhere in the
 * loop (residual, Step 1 and the Schur bound); Siddon with step1_eq6 is the projector and
 * backprojector pair the paper runs. */
typedef struct {
    double lambda;          /* TV weight, >= 0 (1/mu of Eq. 2) */
    const int *iters;       /* iters[l]: outer iterations at level l (l = 0 finest), params.levels entries */
    int levels;             /* levels to run, 1 .. plan levels */
    double step;            /* t (= mu/beta of Algorithm A1); <= 0: Schur bound per level */
    double tv_eps;          /* TV smoothing, 1/mm^2 (default 1e-5) */
    double armijo_c;        /* c of Eq. 5 (default 0.01) */
    double backtrack;       /* alpha of Eq. 5 (default 0.6) */
    double rof_tol;         /* relative-decrease stop of Step 2 (default 1e-3) */
    int rof_max_iter;       /* default 50 */
    int rof_max_backtrack;  /* default 30 */
    const int *replay;      /* NULL, or a forced decision trace (a test hook for FP32 ties): replay_len
                             * records of 2 ints, one per ROF iteration in order: the backtracking
                             * exponent m (-1: the search finds no step) and 1 when that iteration
                             * ends Step 2 (0: Step 2 goes on), taken in place of the device's
                             * Armijo and stop decisions; used up first, then free running */
    int replay_len;
    int step1_eq6;          /* 0 (default): Step 1 uses the exact P^T; 1: the Eq. 6 backprojector
                             * (cbct_backproject_eq6) applied to P f - Y, with the same step */
    double conv_tol;        /* > 0: "until convergence" per level (Section II.C.3): a level stops at
                             * the first k >= 1 with |E(f_k) - E(f_k-1)| <= conv_tol E(f_k-1), iters[l]
                             * being the upper bound (one more stream synchronisation per outer
                             * iteration); 0 (default): exactly iters[l] iterations */
    int projector;          /* 0 (default): trilinear P and its adjoint; 1: Siddon P_s and P_s^T (the
                             * workspace then holds the P_s^T profile tables of the largest level,
                             * cbct_adjoint_siddon_workspace_size); other values: INVALID_ARG */
} cbct_solve_params;

/* Optional diagnostics; arrays are caller-owned and may be NULL (lengths may exceed capacities:
 * the extra records are dropped). */
typedef struct {
    int *trace;             /* 4 ints per ROF iteration: level, outer, inner, m (m = -1: no step) */
    int trace_cap;
    int trace_len;
    double *rof_e;          /* 3 doubles per ROF iteration: E_R(u), E_R at the last tested step, mean(d^2) */
    double *energy;         /* E(f_k), k = 0..iters[l], per level from the coarsest */
    int energy_cap;
    int energy_len;
    double t_used[8];       /* t per level */
    double seconds;         /* host wall time of the call */
    int replay_used;        /* replay entries consumed */
} cbct_solve_stats;

void cbct_solve_params_default(cbct_solve_params *params); /* the defaults above, lambda 0.05, 1 level */

/* Device workspace of cbct_reconstruct for these params (bytes). */
cbct_status cbct_reconstruct_workspace_size(const cbct_plan *plan, const cbct_solve_params *params, size_t *bytes);

/* Full reconstruction.  d_y: level-0 projections [n_views][nv][nu]; d_init: NULL or a level-0
 * start volume; d_out: level-0 result [nz][ny][nx]; d_ws: >= cbct_reconstruct_workspace_size
 * bytes, 256-byte aligned, not shared with a concurrent call.  The call steers the ROF loop
 * from the host: once per ROF iteration it waits for the device-side Armijo decision (64 bytes,
 * written into host-mapped memory and polled, or read after synchronising `stream` when polling
 * is unavailable or times out), and it returns when d_out is final.  The plan's Schur-step cache is the
 * only plan state it writes (guarded by a lock).  INVALID_ARG for bad params or workspace;
 * NONFINITE when an energy or the Schur bound is not finite. */
cbct_status cbct_reconstruct(cbct_plan *plan, const cbct_solve_params *params, const float *d_y,
                             const float *d_init, float *d_out, void *d_ws, size_t ws_bytes,
                             cbct_stream_t stream, cbct_solve_stats *stats);

/* Step 2 alone at `level`: d_u = ROF(d_g) with t = params->step (> 0), from u = g. */
cbct_status cbct_tv_prox_workspace_size(const cbct_plan *plan, int level, size_t *bytes);
cbct_status cbct_tv_prox(cbct_plan *plan, int level, const cbct_solve_params *params, const float *d_g,
                         float *d_u, void *d_ws, size_t ws_bytes, cbct_stream_t stream, cbct_solve_stats *stats);

/* Workspace (device bytes) of cbct_tv_energy_grad (fixed-order partial sums). */
cbct_status cbct_tv_energy_grad_workspace_size(const cbct_plan *plan, size_t *bytes);

/* The TV term of the energy (E_1 of Eq. 2, smoothed; forward differences with the boundary
 * conditions of Section II.B: ghost 0 beyond the last x and y sample, ghost = last plane
 * beyond the last z plane).
 * Smoothed TV sum S(f) = sum_voxels sqrt(|D f|^2 + tv_eps^2) (= N_vox R(f)) and its gradient
 * dS/df into d_grad (may be NULL).  h_sum may be NULL; if not, the call synchronises `stream`
 * and writes S.  d_ws: >= cbct_tv_energy_grad_workspace_size bytes, 8-byte aligned. */
cbct_status cbct_tv_energy_grad(cbct_plan *plan, int level, double tv_eps, const float *d_f, float *d_grad,
                                double *h_sum, void *d_ws, size_t ws_bytes, cbct_stream_t stream);

/* cbct_tv_energy_grad without a workspace, for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops that forbid allocation): the same kernels and the same
 * result, with the partial sums in a 256 KB scratch array that the library holds per device
 * until the process ends (set up by cbct_context_create for its device).  Every call on one GPU
 * shares that GPU's scratch: calls that overlap in time on one GPU (other streams, other
 * threads) race and must be ordered by the caller.  The call allocates nothing.  INVALID_ARG for
 * bad arguments, for a plan whose device had no context made, or for a volume whose partial sums
 * would exceed the scratch. */
cbct_status cbct_tv_energy_grad_noalloc(cbct_plan *plan, int level, double tv_eps, const float *d_f, float *d_grad,
                                        double *h_sum, cbct_stream_t stream);

/* Multigrid transfers (Section II.C.3): cell-centred trilinear prolongation of level
 * coarse_level into level coarse_level-1 (3/4 parent + 1/4 neighbour per axis, clamped), and
 * restriction = (1/8) Prol^T from fine_level into fine_level+1.  Detector restriction for
 * level >= 1: block mean over 2^level x 2^level pixels of the level-0 projections. */
cbct_status cbct_prolong(const cbct_plan *plan, int coarse_level, const float *d_c, float *d_f, cbct_stream_t stream);
cbct_status cbct_restrict(const cbct_plan *plan, int fine_level, const float *d_f, float *d_c, cbct_stream_t stream);
cbct_status cbct_bin_detector(const cbct_plan *plan, int level, const float *d_y0, float *d_yl, cbct_stream_t stream);

/* ---- Serving: continuous admission of reconstruction requests ----------------------------
 *
 * A server owns `max_slots` worker slots, each with its own non-blocking HIP stream on the
 * context's device.  Requests (any geometry, any params without replay) queue FIFO;
 * the head starts as soon as a slot is free and (device bytes in use + its bytes) <= the budget,
 * also while other requests run, so admitted solves overlap on the GPU.  A request's bytes are
 * its reconstruction workspace, its plan tables and, for host projections, their device copy.
 * Results are bitwise identical to a solo cbct_reconstruct of the same request.  Device memory
 * is pooled and plans are cached by geometry for the server's lifetime.  All server calls are
 * thread-safe. */
typedef struct cbct_server cbct_server;

/* INVALID_ARG for a NULL context, budget 0 or max_slots outside 1..256. */
cbct_status cbct_server_create(cbct_context *ctx, size_t hbm_budget_bytes, int max_slots, cbct_server **out);

/* Queue one reconstruction.  y: level-0 projections [n_views][nv][nu], device memory (y_on_host = 0,
 * must stay valid until the request is done) or host memory (y_on_host = 1, copied when the
 * request starts); d_out: device volume [nz][ny][nx] written when the request is done.
 * params->iters is copied; the plan is built with detector binning.  INVALID_ARG for an invalid
 * geometry or params (checked here, before queueing), BUDGET when the request alone exceeds the
 * budget. */
cbct_status cbct_server_submit(cbct_server *server, const cbct_geometry_desc *geom, const cbct_solve_params *params,
                               const float *y, int y_on_host, float *d_out, uint64_t *ticket);

/* done = 1 once the request finished; result = its status; latency_s = submit-to-done seconds
 * (host steady clock), -1 while running.  NOT_FOUND for an unknown ticket. */
cbct_status cbct_server_poll(cbct_server *server, uint64_t ticket, int *done, cbct_status *result, double *latency_s);

/* submit, start and done instants (seconds on the host steady clock) of a finished request */
cbct_status cbct_server_request_times(cbct_server *server, uint64_t ticket, double times[3]);

/* Blocks until the queue is empty and no request runs; returns the first failed request's status. */
cbct_status cbct_server_wait_all(cbct_server *server);

/* Device bytes the server holds now and at its peak (its pooled blocks, idle ones included, and
 * its cached plan tables: what it obtained from hipMalloc; never above the budget), running
 * requests, queue length, completed requests.  A simulated server reports its admission charge. */
cbct_status cbct_server_stats(cbct_server *server, size_t *in_use, size_t *peak_in_use, int *running,
                              int *peak_running, int *queued, uint64_t *completed);

/* Work the batch engine has done so far: batched launches and the request items they carried
 * (items / launches > 1 means launches shared by several requests). */
cbct_status cbct_server_batch_stats(cbct_server *server, uint64_t *launches, uint64_t *items);

/* Stops the workers after their current request (queued requests are dropped) and frees the
 * server's device memory and plans. */
void cbct_server_destroy(cbct_server *server);

/* Scheduler test hooks: a server whose requests sleep `seconds` instead of running on the GPU
 * (same admission and slot logic; no device memory is touched). */
cbct_status cbct_server_create_simulated(size_t hbm_budget_bytes, int max_slots, cbct_server **out);
cbct_status cbct_server_submit_simulated(cbct_server *server, const cbct_geometry_desc *geom,
                                         const cbct_solve_params *params, double seconds, uint64_t *ticket);

/* Human-readable name of a status, and the calling thread's last error message. */
const char *cbct_status_string(cbct_status s);
const char *cbct_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CBCT_H */
