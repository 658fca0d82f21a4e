// Serving runtime: continuous admission of reconstruction requests (Algorithm A1 of the paper per
// request) of mixed volume and view counts under an HBM budget, with the admitted solves batched
// into shared kernel launches.
//
// Admission is FIFO: the head of the queue starts when a slot is free and the device bytes the
// server holds (pooled blocks of running requests and cached plan tables) plus the head's bytes
// fit the budget.  Admitted requests join the batch engine at the next outer-iteration boundary,
// so requests that arrive while others run start without waiting for a batch to drain.
//
// A batch engine (one host thread, one stream) advances every admitted request of its size class
// through the same phase sequence of Algorithm A1, one outer iteration per round:
//   residual P of all requests            one batched launch (per projector configuration)
//   Step 1, g = f - kappa P^T r            per request (its own grid and profile workspace)
//   Step 2, the ROF loop                   gated steps of all requests (apply the accepted step,
//                                          gradient, one trial window, decision: four batched
//                                          launches) enqueued two ahead of the decisions; each
//                                          request's passes read its loop state and idle once its
//                                          loop has ended; the host reads one word per request
//                                          and step and drops finished requests from later steps
//                                          (requests of at most 2^16 voxels run their whole loop
//                                          in one work-group instead)
//   Step 3, f = max(u, 0)                  one batched launch
// There are three engines, for volumes up to 2^18.5 voxels, up to 2^21.5 and larger, on their own
// streams: a round costs about as much as its largest request, so requests of similar size share
// rounds, and the classes overlap on the GPU instead of small requests waiting on large ones.
// Each request's work-groups in a batched launch run the solo kernel's body on that request's
// buffers and grid, and its reductions keep the solo partial layout, so every result is bitwise
// the solo cbct_reconstruct result.  Requests whose options the batched phases do not cover (the
// Siddon pair, the Eq. 6 Step 1, the "until convergence" stop) run one at a time on a side
// worker with its own stream, under the same admission and budget.
//
// Device memory comes from a pool of blocks in exact size classes (a freed block is reused only
// by a request of the same class); idle blocks are returned to the device when an allocation
// would otherwise exceed the budget.  Plans are cached by geometry (with their Schur steps) and
// their tables count against the budget; an unused cached plan is evicted when the budget needs
// the room.
//
// A simulated mode runs the same admission logic with timed sleeps instead of GPU work (host-only
// tests of the scheduler).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cbct_internal.h"

namespace {

using clk = std::chrono::steady_clock;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// size class of a pooled block: 1/16 steps of the next power of two
size_t size_class(size_t n) {
    n = align256(std::max<size_t>(n, 256));
    size_t q = 1;
    while (q < n) q <<= 1;
    const size_t step = std::max<size_t>(q / 16, 256);
    return (n + step - 1) / step * step;
}

struct PlanEntry {
    cbct_plan *plan = nullptr;
    size_t bytes = 0;
    int users = 0;
    clk::time_point last_use;
};

struct Request {
    uint64_t ticket = 0;
    cbct_geometry_desc g{};
    std::vector<double> angles;
    cbct_solve_params p{};
    std::vector<int> iters;
    int levels = 1;
    const float *y = nullptr;
    int y_on_host = 0;
    float *d_out = nullptr;
    bool batchable = true;
    int engine = 0;            // size class: the batch engine that runs it
    std::string key;           // plan cache key
    size_t ws_bytes = 0;       // reconstruction workspace (size class)
    size_t y_bytes = 0;        // device copy of host projections (size class), 0 for device input
    size_t plan_bytes = 0;     // tables of its plan when not cached at admission
    size_t bytes = 0;          // admission charge: ws + y + plan tables if new
    double sim_seconds = 0.0;
    clk::time_point t_submit, t_start, t_done;
    cbct_status result = CBCT_OK;
    std::string err;
    bool done = false;
    // engine state
    PlanEntry *pe = nullptr;
    void *ws = nullptr, *yb = nullptr;
    SolveBufs b{};
    const float *yd = nullptr;
    int level = 0, k = 0, slot = -1;
    double t = 0.0;
    float kappa = 0.0f;
    bool small = false;
    bool dev_init = false;  // its device-side Step 2 state (records, replay position, status) is set
    // Step 2 of the current outer iteration: a gated loop ran (Step 3 applies its pending step);
    // the sequence numbers of the steps enqueued for it
    bool pending = false;
    bool fresh = false;  // this outer iteration's loop is its first device-side Step 2
    std::vector<int> seqs;
};

std::string geom_key(const cbct_geometry_desc &g, const std::vector<double> &angles, int levels) {
    std::string k;
    auto put = [&](const void *p, size_t n) { k.append((const char *)p, n); };
    put(&g.nx, sizeof(int) * 3);
    put(&g.hx, sizeof(double) * 3);
    put(&g.nu, sizeof(int) * 2);
    put(&g.pu, sizeof(double) * 4);
    put(&g.n_views, sizeof(int));
    put(&g.sample_ratio, sizeof(double));
    put(&levels, sizeof(int));
    if (!angles.empty()) put(angles.data(), sizeof(double) * angles.size());
    return k;
}

// reconstruction workspace bytes for a geometry, as cbct_reconstruct_workspace_size computes it
// (an upper bound: the adjoint profiles are counted at the grid support's diagonal)
size_t estimate_ws(const cbct_geometry_desc &g, int levels, const std::vector<int> &iters, int projector,
                   int rof_max_iter) {
    const size_t nvox = (size_t)g.nx * g.ny * g.nz, nray = (size_t)g.n_views * g.nu * g.nv;
    size_t b = 5 * align256(4 * nvox) + align256(4 * std::max(nray, nvox));
    for (int l = 1; l < levels; l++) b += align256(4 * (nray >> (2 * l)));
    size_t parts = (size_t)CBCT_RED_BLOCKS * (3 + 2 * CBCT_TRIALS);
    parts = std::max(parts, (size_t)g.n_views * g.nu);
    b += align256(8 * parts) + align256(8 * 64);
    size_t zmax = 0;
    long rec = 0;
    for (int l = 0; l < levels; l++) {
        const int nx = g.nx >> l, ny = g.ny >> l, nz = g.nz >> l, nu = g.nu >> l;
        const double hx = g.hx * (1 << l), hy = g.hy * (1 << l);
        const double dtau = (g.sample_ratio > 0 ? g.sample_ratio : 1.0) * std::min(hx, hy);
        const double diag = std::sqrt(std::pow((nx + 2) * hx, 2) + std::pow((ny + 2) * hy, 2));
        const size_t zf = (size_t)g.n_views * nu * (((size_t)std::ceil(diag / dtau) + 4) * (size_t)nz + 32) + 64 +
                          (size_t)cbct_adj_vsplit(nx, ny, nz, g.n_views) * nx * ny * nz;
        // the Siddon pair's profile tables instead: (nx + ny + 3) pieces x nz cells per line
        const size_t lines = (size_t)g.n_views * nu;
        const size_t zs = align256(lines * (size_t)(nx + ny + 3) * nz * 4) / 4 + lines * 4;
        zmax = std::max(zmax, projector == 1 ? zs : zf);
        rec = std::max(rec, (long)std::max(iters[l], 1) * rof_max_iter);
    }
    b += align256(4 * zmax);
    int slots = 0;
    for (int l = 0; l < levels; l++) slots += iters[l] + 1;
    b += align256(16 * (size_t)std::max(slots, 1)) + align256(sizeof(RofControl));
    b += align256(sizeof(RofLog)) + align256(sizeof(RofGate)) +
         align256(sizeof(RofRecord) * (size_t)std::max<long>(std::min(rec, 1L << 24), 1)) + 256;
    return b;
}

// device bytes of a plan's tables (all levels), as plan creation allocates them
size_t estimate_plan_bytes(const cbct_geometry_desc &g, int levels) {
    size_t b = 0;
    for (int l = 0; l < levels; l++) {
        const size_t nu = (size_t)(g.nu >> l), cols = (size_t)g.n_views * nu;
        b += align256(sizeof(ColParams) * cols) + align256(sizeof(ViewParams) * g.n_views) +
             align256(sizeof(SidCol) * cols) + align256(sizeof(ZIndex) * cols);
    }
    return b;
}

}  // namespace

struct cbct_server {
    cbct_context ctx;  // the device the server works on (a copy: the caller's context may go first)
    bool simulated = false;
    size_t budget = 0;
    int max_slots = 1;
    std::mutex mu;  // guards everything below
    std::condition_variable cv_work, cv_done, cv_side;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
    size_t held = 0;                 // running requests' blocks + cached plan tables
    size_t owned = 0, plan_total = 0;  // device bytes allocated: pool blocks (idle included), plans
    size_t peak_device = 0;
    int running = 0, peak_running = 0;
    uint64_t next_ticket = 1, completed = 0;
    bool stop = false;
    std::vector<Request *> admitted[3];  // handed to an engine, not yet set up
    Request *side_job = nullptr;
    std::thread engines[3], side;
    std::multimap<size_t, void *> free_blocks;  // idle pool blocks by size class
    std::map<std::string, PlanEntry> plans;
    std::vector<bool> slot_used;
    RofControl *mirror_host = nullptr, *mirror_dev = nullptr;  // host-mapped decision records
    std::atomic<int> seq{0};  // sequence numbers of the gated decisions' words
    // counters of the batched phases (for tests and reports)
    std::atomic<uint64_t> batched_launches{0}, batched_items{0};
};

namespace {

void note_device(cbct_server *s) { s->peak_device = std::max(s->peak_device, s->owned + s->plan_total); }

// (mu held) give back the least recently used cached plans that no running request uses until
// `fits()` holds or none is left
// (`keep`: a plan the caller is about to use, never evicted)
template <class F>
void evict_plans(cbct_server *s, F fits, const std::string *keep = nullptr) {
    while (!fits()) {
        auto victim = s->plans.end();
        for (auto q = s->plans.begin(); q != s->plans.end(); ++q)
            if (q->second.users == 0 && q->second.plan && !(keep && q->first == *keep) &&
                (victim == s->plans.end() || q->second.last_use < victim->second.last_use))
                victim = q;
        if (victim == s->plans.end()) return;
        DeviceGuard dg(s->ctx.device);
        cbct_plan_destroy(victim->second.plan);
        s->plan_total -= victim->second.bytes;
        s->held -= victim->second.bytes;
        s->plans.erase(victim);
    }
}

// (mu held) a block of exactly size class n: an idle one, or a new one; idle blocks, then unused
// cached plans, are released while a new allocation would take the server past its budget
void *pool_get(cbct_server *s, size_t n) {
    auto it = s->free_blocks.find(n);
    if (it != s->free_blocks.end()) {
        void *p = it->second;
        s->free_blocks.erase(it);
        return p;
    }
    DeviceGuard dg(s->ctx.device);
    while (s->owned + s->plan_total + n > s->budget && !s->free_blocks.empty()) {
        auto big = std::prev(s->free_blocks.end());
        hipFree(big->second);
        s->owned -= big->first;
        s->free_blocks.erase(big);
    }
    evict_plans(s, [&] { return s->owned + s->plan_total + n <= s->budget; });
    void *p = nullptr;
    if (hipMalloc(&p, n) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    s->owned += n;
    note_device(s);
    return p;
}

void pool_put(cbct_server *s, void *p, size_t n) {
    if (p) s->free_blocks.emplace(n, p);
}

// (mu not held) the request's plan: cached, or built and cached (its bytes were charged at admission)
cbct_status acquire_plan(cbct_server *s, Request *r) {
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->plans.find(r->key);
        if (it != s->plans.end() && it->second.plan) {
            it->second.users++;
            it->second.last_use = clk::now();
            r->pe = &it->second;
            if (r->plan_bytes) {  // charged for a plan that another request built meanwhile
                s->held -= r->plan_bytes;
                r->bytes -= r->plan_bytes;
                r->plan_bytes = 0;
            }
            return CBCT_OK;
        }
    }
    cbct_plan *p = nullptr;
    cbct_geometry_desc g = r->g;
    g.angles = r->angles.empty() ? nullptr : r->angles.data();
    cbct_status st = cbct_plan_create(&s->ctx, &g, r->levels, 1, &p);
    if (st) return st;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->plans.find(r->key);
    if (it != s->plans.end() && it->second.plan) {  // the other worker built it meanwhile
        cbct_plan_destroy(p);
        it->second.users++;
        it->second.last_use = clk::now();
        r->pe = &it->second;
        s->held -= r->plan_bytes;
        r->bytes -= r->plan_bytes;
        r->plan_bytes = 0;
        return CBCT_OK;
    }
    PlanEntry &e = s->plans[r->key];
    e.plan = p;
    e.bytes = r->plan_bytes;
    if (!e.bytes) {
        // charged nothing at submit (the plan was cached then and has been evicted since): charge
        // its tables now
        e.bytes = estimate_plan_bytes(r->g, r->levels);
        s->held += e.bytes;
    }
    e.users = 1;
    e.last_use = clk::now();
    s->plan_total += e.bytes;
    note_device(s);
    r->pe = &e;
    // the plan's bytes now belong to the cache (still held), not to the request
    r->bytes -= r->plan_bytes;
    r->plan_bytes = 0;
    return CBCT_OK;
}

void admit(cbct_server *s);

// (mu held) finish a request: release its blocks and its hold on the plan, then admit what fits
void release(cbct_server *s, Request *r) {
    pool_put(s, r->ws, r->ws_bytes);
    pool_put(s, r->yb, r->y_bytes);
    r->ws = r->yb = nullptr;
    if (r->pe) {
        r->pe->users--;
        r->pe->last_use = clk::now();
        r->pe = nullptr;
    }
    if (r->slot >= 0) s->slot_used[r->slot] = false;
    s->held -= r->bytes;
    s->running--;
    r->t_done = clk::now();
    r->done = true;
    s->completed++;
    admit(s);
}

// (mu not held) device state of an admitted request: plan, workspace, projections, start volume
cbct_status setup(cbct_server *s, Request *r, hipStream_t stream) {
    cbct_status st = acquire_plan(s, r);
    if (st) return st;
    size_t need = 0;
    r->p.iters = r->iters.data();
    if ((st = cbct_reconstruct_workspace_size(r->pe->plan, &r->p, &need))) return st;
    if (need > r->ws_bytes)
        return cbct_set_error(CBCT_ERR_INTERNAL, "server: workspace %zu bytes exceeds its admission estimate %zu",
                              need, r->ws_bytes);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ws = pool_get(s, r->ws_bytes);
        if (r->ws && r->y_on_host) r->yb = pool_get(s, r->y_bytes);
    }
    if (!r->ws || (r->y_on_host && !r->yb))
        return cbct_set_error(CBCT_ERR_OUT_OF_MEMORY, "server: device memory for request %llu",
                              (unsigned long long)r->ticket);
    r->yd = r->y;
    if (r->y_on_host) {
        CBCT_HIP(hipMemcpyAsync(r->yb, r->y, sizeof(float) * (size_t)r->g.n_views * r->g.nu * r->g.nv,
                                hipMemcpyHostToDevice, stream));
        r->yd = (const float *)r->yb;
    }
    return CBCT_OK;
}

// ---------------------------------------------------------------- side worker (unbatched)
void side_main(cbct_server *s) {
    hipSetDevice(s->ctx.device);
    hipStream_t stream = nullptr;
    hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_side.wait(lk, [&] { return s->stop || s->side_job; });
            if (!s->side_job) break;
            r = s->side_job;
        }
        cbct_status st = setup(s, r, stream);
        if (!st)
            st = cbct_reconstruct(r->pe->plan, &r->p, r->yd, nullptr, r->d_out, r->ws, r->ws_bytes,
                                  (cbct_stream_t)stream, nullptr);
        if (!st && hipStreamSynchronize(stream) != hipSuccess) st = cbct_set_error(CBCT_ERR_HIP, "server: stream sync");
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (st) {
                r->result = st;
                r->err = cbct_last_error();
            }
            s->side_job = nullptr;
            release(s, r);
        }
        s->cv_work.notify_all();
        s->cv_side.notify_all();
        s->cv_done.notify_all();
    }
    if (stream) hipStreamDestroy(stream);
}

// ---------------------------------------------------------------- batch engine
// level start of request r: binned projections, start volume (level transitions prolong), Schur
// step, kappa, projector layout of f
cbct_status start_level(Request *r, hipStream_t s, bool first) {
    cbct_plan *P = r->pe->plan;
    const Level &L = P->lv[r->level];
    cbct_status st;
    if (first) {
        if ((st = cbct_launch_fill(r->b.f, L.nvox(), 0.0f, s))) return st;
    } else {
        if ((st = cbct_launch_prolong(P->lv[r->level + 1], r->b.f, r->b.u, s))) return st;
        std::swap(r->b.f, r->b.u);
    }
    if (r->level > 0) {
        if ((st = cbct_launch_bin(P->lv[0], 1 << r->level, r->yd, r->b.ypyr[r->level], s))) return st;
    }
    double t = r->p.step;
    if (!(t > 0.0) && (st = cbct_solve_schur(P, r->level, 0, r->b, s, &t))) return st;
    r->t = t;
    r->kappa = (float)(t * 2.0 * (double)L.nvox() / (double)L.nray());
    r->small = L.nvox() <= CBCT_SMALL_ROF_VOX && r->b.rec_cap > 0;
    r->k = 0;
    return cbct_launch_to_columns(L, r->b.f, r->b.ft, s);
}

// after outer iteration k of its level: next level, or done (the result copied out)
cbct_status advance(Request *r, hipStream_t s, bool *finished) {
    *finished = false;
    cbct_status st;
    while (r->k >= r->iters[r->level]) {
        if (r->level == 0) {
            const Level &L0 = r->pe->plan->lv[0];
            CBCT_HIP(hipMemcpyAsync(r->d_out, r->b.f, sizeof(float) * L0.nvox(), hipMemcpyDeviceToDevice, s));
            *finished = true;
            return CBCT_OK;
        }
        r->level--;
        if ((st = start_level(r, s, false))) return st;
    }
    return CBCT_OK;
}

const float *level_y(const Request *r) { return r->level > 0 ? r->b.ypyr[r->level] : r->yd; }

// one outer iteration of Algorithm A1 for every request in `act` (all at k < iters[level])
cbct_status round_(cbct_server *s, std::vector<Request *> &act, hipStream_t st_) {
    cbct_status st;
    const int n = (int)act.size();
    // residual r = P f - Y_l with its FP64 sum-of-squares partials
    std::vector<FwdReq> fw(n);
    for (int q = 0; q < n; q++) {
        Request *r = act[q];
        fw[q] = FwdReq{&r->pe->plan->lv[r->level], r->b.ft, level_y(r), r->b.r, r->b.part};
    }
    if ((st = cbct_launch_forward_batch(fw.data(), n, st_))) return st;
    s->batched_launches++;
    s->batched_items += n;
    // Step 1: g = f - kappa P^T r, also into the ROF start u
    std::vector<AdjReq> ad(n);
    for (int q = 0; q < n; q++) {
        Request *r = act[q];
        ad[q] = AdjReq{&r->pe->plan->lv[r->level], r->b.r, r->b.f, r->kappa, r->b.g, r->b.u, r->b.z};
    }
    int nl = 0, ni = 0;
    if ((st = cbct_launch_adjoint_batch(ad.data(), n, st_, &nl, &ni))) return st;
    s->batched_launches += nl;
    s->batched_items += ni;
    // Step 2: the small requests ran their loop in one work-group above; the others run gated
    // steps in shared launches (see cbct_launch_rof_step_gated_batch), AHEAD steps in front of
    // the decisions, and leave the batch when a decision ends their loop
    constexpr int AHEAD = 2;
    std::vector<Request *> rof;
    for (Request *r : act) {
        r->pending = false;
        if (r->small) {
            const Level &L = r->pe->plan->lv[r->level];
            const cbct_solve_params &p = r->p;
            if ((st = cbct_launch_rof_small(L, p.tv_eps, r->b.u, r->b.g, r->b.d, p.lambda, r->t, p.armijo_c,
                                            p.backtrack, p.rof_tol, p.rof_max_iter, p.rof_max_backtrack, nullptr, 0, 0,
                                            r->b.sst, nullptr, r->b.rec_cap, r->level, r->k, !r->dev_init, st_)))
                return st;
            r->dev_init = true;
            continue;
        }
        if (r->p.rof_max_iter > 0) rof.push_back(r);
    }
    if (!rof.empty()) {
        // new loops: their first step's decision starts each loop's state, and a request's records
        // and replay position (unused here) the first time it runs a device-side Step 2
        std::vector<char> fresh(rof.size());
        for (size_t q = 0; q < rof.size(); q++) {
            fresh[q] = !rof[q]->dev_init;
            rof[q]->dev_init = true;
        }
        long max_steps = 0;
        for (Request *r : rof) {
            r->pending = true;  // the clamp applies the last decision's step if it accepted one
            r->seqs.clear();
            max_steps = std::max(max_steps, (long)r->p.rof_max_iter * (2 + r->p.rof_max_backtrack / CBCT_TRIALS));
        }
        std::vector<Request *> active = rof;
        for (size_t q = 0; q < rof.size(); q++) rof[q]->fresh = fresh[q] != 0;
        std::vector<const Level *> lv;
        std::vector<RofStepArgs> args;
        long issued = 0, known = 0;
        while (!active.empty()) {
            while (issued < max_steps && issued < known + AHEAD) {
                lv.clear();
                args.clear();
                for (Request *r : active) {
                    const Level &L = r->pe->plan->lv[r->level];
                    RofStepArgs a{};
                    a.eps = r->p.tv_eps;
                    a.lambda = r->p.lambda;
                    a.t = r->t;
                    a.c_armijo = r->p.armijo_c;
                    a.alpha = r->p.backtrack;
                    a.tol = r->p.rof_tol;
                    a.max_iter = r->p.rof_max_iter;
                    a.max_bt = r->p.rof_max_backtrack;
                    a.u = r->b.u;
                    a.g = r->b.g;
                    a.d = r->b.d;
                    a.part = r->b.part;
                    a.sums = r->b.sums;
                    a.ctl = r->b.ctl;
                    a.gate = r->b.gate;
                    a.st = r->b.sst;
                    a.rec_cap = r->b.rec_cap;
                    a.level = r->level;
                    a.outer = r->k;
                    a.mirror = s->mirror_dev ? &s->mirror_dev[r->slot].pad : nullptr;
                    a.seq = (s->seq.fetch_add(1) + 1) & CBCT_GATE_SEQ_MASK;
                    a.first = issued == 0 ? 1 : 0;
                    a.init_state = (issued == 0 && r->fresh) ? 1 : 0;
                    r->seqs.push_back(a.seq);
                    lv.push_back(&L);
                    args.push_back(a);
                }
                if ((st = cbct_launch_rof_step_gated_batch(lv.data(), args.data(), (int)args.size(), st_))) return st;
                const int nl = issued == 0 ? 3 : 4;  // the first step launches no update
                s->batched_launches += nl;
                s->batched_items += nl * args.size();
                issued++;
            }
            if (known >= issued) break;  // every step a loop can take has run
            // the decisions of step `known` (or later ones) of every active request
            std::vector<int> words(active.size(), 0);
            if (s->mirror_host) {
                for (size_t q = 0; q < active.size(); q++) {
                    Request *r = active[q];
                    const volatile int *p = &s->mirror_host[r->slot].pad;
                    const int want = r->seqs[known];  // every active request is in every step so far
                    const auto t0 = clk::now();
                    bool seen = false;
                    for (int spin = 0;; spin++) {
                        const int w = *p;
                        if ((((w >> 2) - want) & CBCT_GATE_SEQ_MASK) < (CBCT_GATE_SEQ_MASK >> 1)) {
                            words[q] = w;
                            seen = true;
                            break;
                        }
                        if ((spin & 1023) == 1023 && clk::now() - t0 > std::chrono::milliseconds(20)) break;
                    }
                    if (!seen) {
                        CBCT_HIP(hipStreamSynchronize(st_));
                        words[q] = *p;
                    }
                }
            } else {
                // no host-mapped words: read the loop states after the enqueued steps
                CBCT_HIP(hipStreamSynchronize(st_));
                for (size_t q = 0; q < active.size(); q++) {
                    RofGate gs;
                    RofLog ss;
                    CBCT_HIP(hipMemcpy(&gs, active[q]->b.gate, sizeof(gs), hipMemcpyDeviceToHost));
                    CBCT_HIP(hipMemcpy(&ss, active[q]->b.sst, sizeof(ss), hipMemcpyDeviceToHost));
                    words[q] = cbct_gate_word(0, ss.status ? 1 : 0, gs.run);
                }
            }
            std::vector<Request *> next;
            for (size_t q = 0; q < active.size(); q++) {
                if (words[q] & 2)
                    return cbct_set_error(CBCT_ERR_NONFINITE, "ROF energy is not finite (request %llu)",
                                          (unsigned long long)active[q]->ticket);
                if (words[q] & 1) next.push_back(active[q]);
            }
            active.swap(next);
            known++;
        }
    }
    // Step 3 (with the last ROF update when it is pending)
    std::vector<ClampReq> cl(n);
    for (int q = 0; q < n; q++) {
        Request *r = act[q];
        cl[q] = ClampReq{&r->pe->plan->lv[r->level], r->b.u, r->pending ? r->b.d : nullptr,
                         r->pending ? r->b.ctl : nullptr, r->b.f, r->b.ft};
    }
    if ((st = cbct_launch_clamp_batch(cl.data(), n, st_))) return st;
    s->batched_launches++;
    s->batched_items += n;
    return CBCT_OK;
}

void fail(cbct_server *s, Request *r, cbct_status st) {
    std::lock_guard<std::mutex> lk(s->mu);
    r->result = st;
    r->err = cbct_last_error();
    release(s, r);
}

void engine_main(cbct_server *s, int cls) {
    hipSetDevice(s->ctx.device);
    hipStream_t stream = nullptr;
    hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    std::vector<Request *> act;
    for (;;) {
        std::vector<Request *> fresh;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->admitted[cls].empty() || !act.empty(); });
            if (s->stop && s->admitted[cls].empty() && act.empty()) break;
            fresh.swap(s->admitted[cls]);
        }
        bool any_done = false;
        for (Request *r : fresh) {
            cbct_status st = setup(s, r, stream);
            if (!st) {
                r->b = cbct_solve_carve(r->pe->plan, &r->p, r->ws);
                r->level = r->levels - 1;
                st = start_level(r, stream, true);
            }
            bool fin = false;
            if (!st) st = advance(r, stream, &fin);  // levels with no iterations
            if (st) {
                fail(s, r, st);
                any_done = true;
                continue;
            }
            if (fin) {
                if (hipStreamSynchronize(stream) != hipSuccess) (void)hipGetLastError();
                std::lock_guard<std::mutex> lk(s->mu);
                release(s, r);
                any_done = true;
                continue;
            }
            act.push_back(r);
        }
        if (!act.empty()) {
            cbct_status st = round_(s, act, stream);
            std::vector<Request *> keep, finished;
            for (Request *r : act) {
                bool fin = false;
                if (!st) {
                    r->k++;
                    st = advance(r, stream, &fin);
                }
                if (st) {
                    // a failed round takes down the requests it carried (their state is unknown)
                    if (hipStreamSynchronize(stream) != hipSuccess) (void)hipGetLastError();
                    fail(s, r, st);
                    any_done = true;
                    continue;
                }
                (fin ? finished : keep).push_back(r);
            }
            if (!finished.empty()) {
                cbct_status sst = hipStreamSynchronize(stream) == hipSuccess ? CBCT_OK : CBCT_ERR_HIP;
                for (Request *r : finished) {
                    if (!sst && r->dev_init) {
                        RofLog ss;
                        if (hipMemcpy(&ss, r->b.sst, sizeof(ss), hipMemcpyDeviceToHost) == hipSuccess && ss.status)
                            sst = cbct_set_error(CBCT_ERR_NONFINITE, "ROF energy is not finite (device-side Step 2)");
                    }
                    std::lock_guard<std::mutex> lk(s->mu);
                    if (sst) {
                        r->result = sst;
                        r->err = cbct_last_error();
                    }
                    release(s, r);
                }
                any_done = true;
            }
            act.swap(keep);
        }
        if (any_done) {
            s->cv_work.notify_all();
            s->cv_side.notify_all();
            s->cv_done.notify_all();
        }
    }
    if (stream) hipStreamDestroy(stream);
}

// ---------------------------------------------------------------- admission
// (mu held) admit queue heads while a slot and the budget allow
void admit(cbct_server *s) {
    while (!s->queue.empty() && !s->stop) {
        Request *h = s->queue.front();
        if (s->running >= s->max_slots) break;
        // cached plans nobody uses make room for the head (its own plan is charged to it while new)
        if (!s->simulated) evict_plans(s, [&] { return s->held + h->bytes <= s->budget; }, &h->key);
        if (s->held + h->bytes > s->budget) break;
        if (s->simulated) {
            // no device work: the request holds its slot and bytes for its service time
        } else if (!h->batchable) {
            if (s->side_job) break;  // FIFO: the head waits for the side worker
        }
        s->queue.pop_front();
        s->held += h->bytes;
        if (s->simulated) s->peak_device = std::max(s->peak_device, s->held);  // its stand-in for device bytes
        s->running++;
        s->peak_running = std::max(s->peak_running, s->running);
        h->t_start = clk::now();
        if (s->simulated) continue;
        for (int q = 0; q < (int)s->slot_used.size(); q++)
            if (!s->slot_used[q]) {
                s->slot_used[q] = true;
                h->slot = q;
                break;
            }
        if (h->batchable) s->admitted[h->engine].push_back(h);
        else s->side_job = h;
    }
}

// simulated mode: a timer thread finishes requests after their service time
void sim_main(cbct_server *s) {
    std::vector<Request *> run;
    for (;;) {
        std::unique_lock<std::mutex> lk(s->mu);
        admit(s);
        for (auto &kv : s->all)
            if (!kv.second->done && kv.second->t_start != clk::time_point() &&
                std::find(run.begin(), run.end(), kv.second.get()) == run.end())
                run.push_back(kv.second.get());
        const auto now = clk::now();
        bool any = false;
        for (auto it = run.begin(); it != run.end();) {
            Request *r = *it;
            if (now - r->t_start >= std::chrono::duration<double>(r->sim_seconds)) {
                s->held -= r->bytes;
                s->running--;
                r->t_done = now;
                r->done = true;
                s->completed++;
                it = run.erase(it);
                any = true;
            } else {
                ++it;
            }
        }
        if (any) {
            admit(s);
            s->cv_done.notify_all();
            continue;
        }
        if (s->stop && run.empty()) break;
        s->cv_work.wait_for(lk, std::chrono::milliseconds(1));
        if (s->stop && run.empty() && s->queue.empty()) break;
    }
}

cbct_status server_create(const cbct_context *ctx, size_t budget, int max_slots, bool sim, cbct_server **out) {
    if (!out || budget == 0 || max_slots < 1 || max_slots > 256)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_create: need out, budget > 0 and 1..256 slots");
    if (!sim && !ctx) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_create: NULL context");
    auto *s = new (std::nothrow) cbct_server();
    if (!s) return cbct_set_error(CBCT_ERR_OUT_OF_MEMORY, "server_create: host allocation");
    s->simulated = sim;
    s->budget = budget;
    s->max_slots = max_slots;
    s->slot_used.assign(max_slots, false);
    if (!sim) {
        s->ctx = *ctx;
        DeviceGuard dg(s->ctx.device);
        void *h = nullptr, *d = nullptr;
        if (hipHostMalloc(&h, sizeof(RofControl) * max_slots, hipHostMallocMapped | hipHostMallocCoherent) ==
                hipSuccess &&
            hipHostGetDevicePointer(&d, h, 0) == hipSuccess) {
            s->mirror_host = (RofControl *)h;
            s->mirror_dev = (RofControl *)d;
            std::memset(h, 0, sizeof(RofControl) * max_slots);
        } else {
            (void)hipGetLastError();  // decisions are then copied back instead
        }
        for (int c = 0; c < 3; c++) s->engines[c] = std::thread(engine_main, s, c);
        s->side = std::thread(side_main, s);
    } else {
        s->engines[0] = std::thread(sim_main, s);
    }
    *out = s;
    return CBCT_OK;
}

cbct_status submit(cbct_server *s, const cbct_geometry_desc *g, const cbct_solve_params *p, const float *y,
                   int y_on_host, float *d_out, double sim_seconds, uint64_t *ticket) {
    if (!s || !g || !p || !ticket) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit: NULL argument");
    if (!s->simulated && (!y || !d_out)) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit: NULL data");
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || g->nu <= 0 || g->nv <= 0 || g->n_views <= 0 || !(g->hx > 0) ||
        !(g->hy > 0) || !(g->hz > 0) || !(g->pu > 0) || !(g->pv > 0) || !(g->sdd > g->sad) || !(g->sad > 0))
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit: invalid geometry");
    if (p->levels < 1 || p->levels > 8 || !p->iters)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit: invalid params.levels or iters");
    for (int l = 0; l < p->levels; l++)
        if (p->iters[l] < 0 || p->iters[l] > 100000)
            return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit: iters[%d] out of range", l);
    const int f = 1 << (p->levels - 1);
    if (g->nx % f || g->ny % f || g->nz % f || g->nu % f || g->nv % f)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit: dims not divisible by 2^(levels-1)");
    if (p->replay) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit: replay is a test-only solve option");
    if (p->projector != 0 && p->projector != 1)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit: projector %d is neither 0 nor 1", p->projector);
    auto r = std::make_unique<Request>();
    r->g = *g;
    if (g->angles) r->angles.assign(g->angles, g->angles + g->n_views);
    r->g.angles = nullptr;
    r->p = *p;
    r->iters.assign(p->iters, p->iters + p->levels);
    r->p.iters = r->iters.data();
    r->levels = p->levels;
    r->y = y;
    r->y_on_host = y_on_host;
    r->d_out = d_out;
    r->sim_seconds = sim_seconds;
    r->batchable = p->projector == 0 && p->step1_eq6 == 0 && !(p->conv_tol > 0.0);
    const long nvox = (long)g->nx * g->ny * g->nz;
    r->engine = nvox <= 370000 ? 0 : nvox <= 3000000 ? 1 : 2;
    r->key = geom_key(r->g, r->angles, r->levels);
    r->ws_bytes = size_class(estimate_ws(*g, p->levels, r->iters, p->projector, p->rof_max_iter));
    r->y_bytes = y_on_host ? size_class(sizeof(float) * (size_t)g->n_views * g->nu * g->nv) : 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->plan_bytes = s->plans.count(r->key) ? 0 : estimate_plan_bytes(*g, p->levels);
    }
    r->bytes = r->ws_bytes + r->y_bytes + r->plan_bytes;
    if (r->bytes > s->budget)
        return cbct_set_error(CBCT_ERR_BUDGET, "server_submit: request needs %zu bytes, budget %zu", r->bytes, s->budget);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit: server is shutting down");
        r->ticket = s->next_ticket++;
        r->t_submit = clk::now();
        *ticket = r->ticket;
        s->queue.push_back(r.get());
        s->all.emplace(r->ticket, std::move(r));
        admit(s);
    }
    s->cv_work.notify_all();
    s->cv_side.notify_all();
    return CBCT_OK;
}

}  // namespace

extern "C" cbct_status cbct_server_create(cbct_context *ctx, size_t hbm_budget_bytes, int max_slots,
                                          cbct_server **out) {
    return server_create(ctx, hbm_budget_bytes, max_slots, false, out);
}

extern "C" cbct_status cbct_server_create_simulated(size_t hbm_budget_bytes, int max_slots, cbct_server **out) {
    return server_create(nullptr, hbm_budget_bytes, max_slots, true, out);
}

extern "C" cbct_status cbct_server_submit(cbct_server *s, const cbct_geometry_desc *g, const cbct_solve_params *p,
                                          const float *y, int y_on_host, float *d_out, uint64_t *ticket) {
    if (s && s->simulated) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit: simulated server");
    return submit(s, g, p, y, y_on_host, d_out, 0.0, ticket);
}

extern "C" cbct_status cbct_server_submit_simulated(cbct_server *s, const cbct_geometry_desc *g,
                                                    const cbct_solve_params *p, double seconds, uint64_t *ticket) {
    if (!s || !s->simulated) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit_simulated: not simulated");
    return submit(s, g, p, nullptr, 0, nullptr, seconds, ticket);
}

extern "C" cbct_status cbct_server_poll(cbct_server *s, uint64_t ticket, int *done, cbct_status *result,
                                        double *latency_s) {
    if (!s || !done) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return cbct_set_error(CBCT_ERR_NOT_FOUND, "server_poll: unknown ticket %llu",
                                                  (unsigned long long)ticket);
    const Request *r = it->second.get();
    *done = r->done ? 1 : 0;
    if (result) *result = r->done ? r->result : CBCT_OK;
    if (latency_s)
        *latency_s = r->done ? std::chrono::duration<double>(r->t_done - r->t_submit).count() : -1.0;
    return CBCT_OK;
}

extern "C" cbct_status cbct_server_request_times(cbct_server *s, uint64_t ticket, double times[3]) {
    if (!s || !times) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_request_times: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return cbct_set_error(CBCT_ERR_NOT_FOUND, "server_request_times: unknown ticket");
    const Request *r = it->second.get();
    if (!r->done) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_request_times: not done");
    const auto epoch = clk::time_point();
    times[0] = std::chrono::duration<double>(r->t_submit - epoch).count();
    times[1] = std::chrono::duration<double>(r->t_start - epoch).count();
    times[2] = std::chrono::duration<double>(r->t_done - epoch).count();
    return CBCT_OK;
}

extern "C" cbct_status cbct_server_wait_all(cbct_server *s) {
    if (!s) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_wait_all: NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->queue.empty() && s->running == 0; });
    for (auto &kv : s->all)
        if (kv.second->result != CBCT_OK)
            return cbct_set_error(kv.second->result, "request %llu failed: %s", (unsigned long long)kv.first,
                                  kv.second->err.c_str());
    return CBCT_OK;
}

extern "C" cbct_status cbct_server_stats(cbct_server *s, size_t *in_use, size_t *peak_in_use, int *running,
                                         int *peak_running, int *queued, uint64_t *completed) {
    if (!s) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_stats: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    // simulated servers allocate nothing: report their admission charge instead
    if (in_use) *in_use = s->simulated ? s->held : s->owned + s->plan_total;
    if (peak_in_use) *peak_in_use = s->peak_device;
    if (running) *running = s->running;
    if (peak_running) *peak_running = s->peak_running;
    if (queued) *queued = (int)s->queue.size();
    if (completed) *completed = s->completed;
    return CBCT_OK;
}

extern "C" cbct_status cbct_server_batch_stats(cbct_server *s, uint64_t *launches, uint64_t *items) {
    if (!s) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_batch_stats: NULL server");
    if (launches) *launches = s->batched_launches.load();
    if (items) *items = s->batched_items.load();
    return CBCT_OK;
}

extern "C" void cbct_server_destroy(cbct_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // queued requests are dropped; running ones finish
        s->queue.clear();
    }
    s->cv_work.notify_all();
    s->cv_side.notify_all();
    for (auto &t : s->engines)
        if (t.joinable()) t.join();
    if (s->side.joinable()) s->side.join();
    if (!s->simulated) {
        DeviceGuard dg(s->ctx.device);
        for (auto &kv : s->plans) cbct_plan_destroy(kv.second.plan);
        for (auto &kv : s->free_blocks) hipFree(kv.second);
        if (s->mirror_host) hipHostFree(s->mirror_host);
    }
    delete s;
}
