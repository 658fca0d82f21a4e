// Internal declarations shared by the libcbct host code and kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "cbct.h"

#include "geometry_tables.h"


struct Level {
    int nx, ny, nz, nu, nv, nviews;
    double hx, hy, hz, pu, pv, sad, sdd, dtau;
    std::vector<double> angles;
    // forward projector table geometry
    int fwd_pad;   // zero cells on either side of the z range in the ray-sample tables
    int fwd_kc;    // samples per table chunk
    int fwd_kr;    // samples per chunk of the run-summing projector (0: its tables do not fit)
    int fwd_tw;    // table rows (z cells incl. padding)
    // adjoint
    AdjArgs adj;
    long z_floats = 0;            // size of the adjoint workspace (profiles + view-group partials)
    int zk_max = 0;               // most samples of one column inside the grid's support
    int adj_vsplit = 1;           // view groups of the adjoint gather
    long adj_part_off = 0;        // float offset of the view-group partial volumes
    ZIndex *d_zix = nullptr;      // [nviews][nu]
    double schur_t = 0.0;         // cached Schur-bound step of the trilinear pair (0: not computed yet)
    double schur_t_siddon = 0.0;  // the same for the Siddon pair
    // device tables
    ColParams *d_cols = nullptr;   // [nviews][nu]
    ViewParams *d_views = nullptr; // [nviews]
    SidCol *d_sid = nullptr;       // [nviews][nu]
    long nvox() const { return (long)nx * ny * nz; }
    long nray() const { return (long)nviews * nv * nu; }
};

// A HIP device the library works on: plans and servers are created on it and keep it.
struct cbct_context {
    int device = 0;
    size_t total_mem = 0;
    char arch[64] = {0};
};

// Makes `device` current for the lifetime of the guard and restores the caller's device.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int device) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != device) (void)hipSetDevice(device);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
    DeviceGuard(const DeviceGuard &) = delete;
    DeviceGuard &operator=(const DeviceGuard &) = delete;
};

struct cbct_plan {
    int device = 0;
    int levels = 1;
    int bin_detector = 1;
    std::vector<Level> lv;
};

// error plumbing (thread-local message)
cbct_status cbct_set_error(cbct_status s, const char *fmt, ...);
cbct_status cbct_hip_error(hipError_t e, const char *what);
#define CBCT_HIP(call)                                          \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return cbct_hip_error(e_, #call); \
    } while (0)

// kernel launchers (each checks its launch)
// work-group size of the run-summing projector for nv detector rows (row pairs split evenly over
// threads, whole waves); *npt: row pairs per thread
int cbct_forward_runs_block(int nv, int *npt);
// chunk of the run-summing projector for nz cells and work-groups of nwaves waves (0: its LDS
// tables do not fit)
int cbct_forward_run_chunk(int nz, int nwaves);
cbct_status cbct_launch_to_columns(const Level &L, const float *vol, float *vol_t, hipStream_t s);
// y_sub == NULL: out = P f.  Otherwise residual mode: out = w * (P f - y_sub) (the ray weight
// applied, ready for the pre-weighted adjoint; plain P f - y_sub when weight_residual is false)
// and partials[view * nu + i] = sum (P f - y_sub)^2.
cbct_status cbct_launch_forward(const Level &L, const float *vol_t, const float *y_sub, float *out,
                                double *partials, hipStream_t s, bool weight_residual = true);
// out = B proj (f_base == NULL) or f_base - kappa B proj, B the Eq. 6 backprojector; out2
// (optional) receives the same volume.
cbct_status cbct_launch_backproject_eq6(const Level &L, const float *proj, const float *f_base, float kappa,
                                        float *out, hipStream_t s, float *out2 = nullptr);
// out = P^T proj (f_base == NULL) or f_base - kappa P^T proj; Zws holds L.z_floats floats; out2
// (optional) receives the same volume.
cbct_status cbct_launch_adjoint(const Level &L, const float *proj, const float *f_base, float kappa,
                                float *out, float *Zws, hipStream_t s, bool preweighted = false,
                                float *out2 = nullptr);
// Siddon pair: out = P_s vol_t (vol_t in the column-major layout), or with y_sub the residual
// out = P_s vol_t - y_sub and partials[view * nu + i] = sum of its squares; out = P_s^T proj, or
// f_base - kappa P_s^T proj.
cbct_status cbct_launch_forward_siddon(const Level &L, const float *vol_t, const float *y_sub, float *out,
                                       double *partials, hipStream_t s);
// P_s^T through per-piece z profiles in ws (cbct_adjoint_siddon_ws_bytes), or the per-cell gather
cbct_status cbct_launch_adjoint_siddon(const Level &L, const float *proj, const float *f_base, float kappa, float *out,
                                       void *ws, hipStream_t s, float *out2 = nullptr);
size_t cbct_adjoint_siddon_ws_bytes(const Level &L);

// ---- solver pieces --------------------------------------------------------------------------
constexpr int CBCT_RED_BLOCKS = 8192;  // work-groups of the fixed-size reduction grids
constexpr int CBCT_TRIALS = 4;         // Armijo step sizes evaluated per trial pass

// The hardware deals the work-groups of a launch round-robin to the 8 XCDs, each with its own L2.
// Remapping the linear work-group index w -> (w mod 8) (G / 8) + w / 8 hands every XCD a
// contiguous range instead, so work-groups that read neighbouring data share one L2 (identity
// unless G is a multiple of 8).
__device__ __forceinline__ int cbct_xcd_remap(int w, int G) {
    return (G & 7) ? w : (w & 7) * (G >> 3) + (w >> 3);
}

// In a batched launch a request's work-groups start at wg0 and number G, both multiples of 8 (the
// launcher pads G): the request's own index of this work-group in the XCD-aware order of a solo
// launch of G work-groups (the XCD is blockIdx.x % 8, and wg0 % 8 == 0).  Indices past the
// request's real count belong to padding work-groups, which return at once.
__device__ __forceinline__ int cbct_batch_local(int wg0, int G) { return cbct_xcd_remap((int)blockIdx.x - wg0, G); }
inline int cbct_batch_pad(int n) { return (n + 7) & ~7; }

// Device-side result of one Armijo search window (read by the host after each ROF iteration).
struct RofControl {
    double e0;       // E_R(u)
    double G;        // mean(d^2)
    double e_trial;  // E_R(u - s d) at the last tested step
    double s;        // last tested step
    int m;           // its backtracking exponent
    int accepted;    // 1: step accepted, -1: no admissible step, 0: search continues at next_m0
    int next_m0;
    int pad;         // in the host-mapped copy: the decision call's sequence number, written last
};

// Step 2 on the device keeps its records, the replay position and a non-finite flag in device
// memory across the outer iterations of a level (read back once per level).  Volumes of at most
// CBCT_SMALL_ROF_VOX voxels run the whole loop in one work-group (for 16^3 and smaller it beats
// launching the passes: 8^3 / 16^3 levels of a low-dose cascade); larger ones run gated chains.
constexpr long CBCT_SMALL_ROF_VOX = 4096;
struct RofLog {
    int n_rec;       // records appended so far (also those beyond the buffer)
    int replay_pos;  // replay records consumed
    int status;      // 1: a non-finite energy stopped the loop
    int pad;
};
struct RofRecord {
    double e0, e_trial, G;
    int level, outer, inner, m;  // m = -1: no admissible step
};
static_assert(sizeof(RofRecord) == 40, "RofRecord layout");

// Step 2 of a larger volume as flag-gated launch chains: the host enqueues steps (apply the last
// accepted step, a new gradient, one trial window, the decision) ahead of the decisions; every
// pass reads this state first and does nothing once the loop has ended or when the step does not
// need it.  The decision kernel updates it; records and the replay position are those of
// RofLog.
struct RofGate {
    int run;      // 1 while the loop continues
    int m0;       // first backtracking exponent of the next trial window
    int apply;    // the next step starts with u -= s d (s of the accepted decision in RofControl)
    int grad;     // the next step computes a new gradient
    int it;       // ROF iteration of the next decision
    int pending;  // the loop ended on an accepted step that is not applied to u
    int pad[2];
};
// host-mapped word a gated decision writes last: (sequence << 2) | (non-finite << 1) | running
__host__ __device__ inline int cbct_gate_word(int seq, int status, int run) { return (seq << 2) | (status << 1) | run; }
constexpr int CBCT_GATE_SEQ_MASK = 0x1fffffff;  // sequence numbers wrap within 29 bits
struct RofStepArgs {
    double eps, lambda, t, c_armijo, alpha, tol;
    int max_iter, max_bt;
    float *u;
    const float *g;
    float *d;
    double *part;  // gradient partials at part, trial partials at part + 3 CBCT_RED_BLOCKS
    double *sums;  // [0..2] gradient sums, [3..] trial sums
    RofControl *ctl;
    RofGate *gate;
    RofLog *st;
    const int *replay;
    int replay_len;
    RofRecord *rec;  // NULL: no records (the count still advances)
    int rec_cap, level, outer;
    int *mirror;  // host-mapped word (device address), or NULL
    int seq;
    int first;       // the loop's first step: no update, ungated passes, the decision starts the state
    int init_state;  // with first: the level's first loop (the records and replay position start too)
    int replay_pos;  // with init_state: the replay position at the level's start
};
cbct_status cbct_launch_rof_step_gated(const Level &L, const RofStepArgs &a, hipStream_t s);
// u -= s d when the gated loop ended on a pending accepted step
cbct_status cbct_launch_axpy_pending(float *u, const float *d, const RofControl *ctl, const RofGate *gate, long n,
                                     hipStream_t s);
cbct_status cbct_launch_rof_small(const Level &L, double eps, float *u, const float *g, float *d, double lambda,
                                  double t, double c_armijo, double alpha, double tol, int max_iter, int max_bt,
                                  const int *replay, int replay_len, int replay_pos, RofLog *st,
                                  RofRecord *rec, int rec_cap, int level, int outer, bool init, hipStream_t s);

int cbct_reduce_blocks(const Level &L);
// Device scratch of cbct_tv_energy_grad_noalloc: a file-scope device array of this size per
// device, its address looked up once per device (with the device current) by context creation.
constexpr size_t CBCT_NOALLOC_SCRATCH_BYTES = 256 * 1024;
constexpr int CBCT_MAX_DEVICES = 64;
cbct_status cbct_noalloc_scratch_init(int device);
void *cbct_noalloc_scratch(int device);  // NULL before cbct_noalloc_scratch_init on that device
cbct_status cbct_launch_tv_grad(const Level &L, double eps, const float *u, const float *g, float *d, double lambda,
                                double t, double *partials, double *sums, hipStream_t s);
cbct_status cbct_launch_tv_energy(const Level &L, double eps, const float *u, double *partials, double *sum,
                                  hipStream_t s);
// trial energies for the M (1 or CBCT_TRIALS) step sizes t alpha^(m0 .. m0+M-1)
cbct_status cbct_launch_tv_trial(const Level &L, double eps, const float *u, const float *d, const float *g,
                                 double t, double alpha, int m0, int M, double *partials, double *sums, hipStream_t s);
cbct_status cbct_launch_rof_decide(const double *sums, int m0, int M, int forced_m, long nvox, double lambda,
                                   double t, double c_armijo, double alpha, int max_bt, RofControl *ctl,
                                   RofControl *mirror, int seq, hipStream_t s);
cbct_status cbct_launch_axpy_step(float *u, const float *d, const RofControl *ctl, long n, hipStream_t s);
cbct_status cbct_launch_sum_rows(const double *part, int nb, int width, double *out, hipStream_t s);

// Buffers of a reconstruction carved from its workspace (cbct_reconstruct's layout).
struct SolveBufs {
    float *f, *ft, *g, *u, *d, *r, *z;
    float *ypyr[8];
    double *part, *sums, *eng;
    RofControl *ctl;
    RofLog *sst;  // Step 2 on the device: records and replay position
    RofGate *gate;       // Step 2 as gated launch chains (larger levels)
    RofRecord *rec;
    int rec_cap;
    int *replay;         // device copy of params.replay (2 ints per record)
    size_t bytes;
};
SolveBufs cbct_solve_carve(const cbct_plan *p, const cbct_solve_params *pr, void *ws);
// Schur-bound step of a level (cached in the plan)
cbct_status cbct_solve_schur(cbct_plan *p, int level, int projector, const SolveBufs &b, hipStream_t s, double *t);

// ---- batched launches (the serving engine): one launch carries the work-groups of several
// requests; each request's work-groups run the solo kernel's body on that request's buffers and
// grid, so its results are bitwise those of a solo launch.
constexpr int CBCT_MAXB = 16;  // requests per batched launch
// one gated Step 2 step of several requests (each with its own level, buffers and loop state)
cbct_status cbct_launch_rof_step_gated_batch(const Level *const *L, const RofStepArgs *a, int n, hipStream_t s);
struct ClampReq {
    const Level *L;
    const float *u, *d;
    const RofControl *ctl;
    float *f, *f_t;
};
cbct_status cbct_launch_clamp_batch(const ClampReq *r, int n, hipStream_t s);
struct FwdReq {
    const Level *L;
    const float *vol_t, *ysub;
    float *out;
    double *partials;
};
// residual P of several requests; requests whose projector configuration differs from the first
// one's go to further launches (same stream)
cbct_status cbct_launch_forward_batch(const FwdReq *r, int n, hipStream_t s);
struct AdjReq {
    const Level *L;
    const float *proj;   // w * (P f - Y) (preweighted)
    const float *fbase;  // out = fbase - kappa P^T proj
    float kappa;
    float *out, *out2;   // out2: a second copy of out (may be null)
    float *Zws;          // the request's adjoint workspace
};
// Step 1 of several requests (cbct_launch_adjoint with preweighted input): one launch each for
// the profiles, the staged gathers and the view-group sums; requests whose depth is not a
// multiple of 32 get launches of their own.  *launches: the number of launches made, *items: the
// number of (request, launch) pairs they carried.
cbct_status cbct_launch_adjoint_batch(const AdjReq *r, int n, hipStream_t s, int *launches, int *items);

// multigrid transfers and small vector kernels
cbct_status cbct_launch_prolong(const Level &coarse, const float *c, float *f, hipStream_t s);
cbct_status cbct_launch_restrict(const Level &coarse, const float *f, float *c, hipStream_t s);
cbct_status cbct_launch_bin(const Level &fine0, int factor, const float *y0, float *yl, hipStream_t s);
// f = max(v, 0) and its column-major copy f_t, v = u, or u - s d when d is given and the decision
// record ctl accepted a step of size s (a ROF update left pending by the loop).
cbct_status cbct_launch_clamp_columns(const Level &L, const float *u, float *f, float *f_t, hipStream_t s,
                                      const float *d = nullptr, const RofControl *ctl = nullptr);
cbct_status cbct_launch_fill(float *x, long n, float v, hipStream_t s);
cbct_status cbct_launch_max(const float *x, long n, double *partials, double *out, hipStream_t s);
