// Serving runtime: reconstruction requests of mixed volume and view counts are admitted as
// worker slots and HBM budget free up, each solve keeps its state (plan tables, workspace,
// projections) on the device, and the admitted solves run concurrently on their own
// non-blocking HIP streams, so their kernels overlap on the GPU.  A request that arrives while
// others run starts as soon as a slot and its memory are available (no batch boundary).
//
// Admission is FIFO: the head of the queue starts when (bytes in use + its bytes) <= budget and
// a slot is free.  Device memory comes from a caching pool (freed blocks are reused and only
// returned at server destruction: hipFree would synchronise the device under running solves);
// plans are cached by geometry, which also keeps their Schur step estimates.
//
// A simulated mode runs the same admission and slot logic with a timed sleep instead of GPU work
// (host-only tests of the scheduler).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
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
    size_t bytes = 0;      // device bytes held while running (workspace + projections copy)
    size_t ws_bytes = 0;
    double sim_seconds = 0.0;
    clk::time_point t_submit, t_start, t_done;
    cbct_status result = CBCT_OK;
    std::string err;
    bool done = false;
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
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t estimate_ws(const cbct_geometry_desc &g, int levels, const std::vector<int> &iters, int projector) {
    const size_t nvox = (size_t)g.nx * g.ny * g.nz, nray = (size_t)g.n_views * g.nu * g.nv;
    size_t b = 5 * align256(4 * nvox) + align256(4 * std::max(nray, nvox));
    for (int l = 1; l < levels; l++) b += align256(4 * (nray >> (2 * l)));
    size_t parts = (size_t)CBCT_RED_BLOCKS * (3 + 2 * CBCT_TRIALS);
    parts = std::max(parts, (size_t)g.n_views * g.nu);
    b += align256(8 * parts) + align256(8 * 64);
    // adjoint workspace, the largest over the levels: profiles (at most grid support diagonal /
    // sample step + 3 samples per column) and the view-group partial volumes
    size_t zmax = 0;
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
    }
    b += align256(4 * zmax);
    int slots = 0;
    for (int l = 0; l < levels; l++) slots += iters[l] + 1;
    b += align256(16 * (size_t)std::max(slots, 1)) + align256(sizeof(RofControl));
    return b;
}

}  // namespace

struct cbct_server {
    cbct_context ctx;  // the device the server works on (a copy: the caller's context may go first)
    bool simulated = false;
    size_t budget = 0;
    int max_slots = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
    size_t in_use = 0, peak_in_use = 0;
    int running = 0, peak_running = 0;
    uint64_t next_ticket = 1, completed = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    // device memory pool and plan cache (guarded by pool_mu)
    std::mutex pool_mu;
    std::multimap<size_t, void *> free_blocks;
    std::vector<void *> owned;
    std::map<std::string, cbct_plan *> plans;
};

namespace {

void *pool_get(cbct_server *s, size_t n) {
    std::lock_guard<std::mutex> lk(s->pool_mu);
    auto it = s->free_blocks.lower_bound(n);
    if (it != s->free_blocks.end() && it->first <= 2 * n) {
        void *p = it->second;
        s->free_blocks.erase(it);
        return p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, n) != hipSuccess) return nullptr;
    s->owned.push_back(p);
    return p;
}

void pool_put(cbct_server *s, void *p, size_t n) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(s->pool_mu);
    s->free_blocks.emplace(n, p);
}

// pooled blocks are tagged with their real size
struct Block {
    void *p = nullptr;
    size_t n = 0;
};

Block block_get(cbct_server *s, size_t n) {
    n = align256(std::max<size_t>(n, 256));
    // round to 1/16 steps of the next power of two so that freed blocks fit later requests
    size_t q = 1;
    while (q < n) q <<= 1;
    const size_t step = std::max<size_t>(q / 16, 256);
    n = (n + step - 1) / step * step;
    return Block{pool_get(s, n), n};
}

cbct_status get_plan(cbct_server *s, Request *r, cbct_plan **out) {
    const std::string key = geom_key(r->g, r->angles, r->levels);
    {
        std::lock_guard<std::mutex> lk(s->pool_mu);
        auto it = s->plans.find(key);
        if (it != s->plans.end()) {
            *out = it->second;
            return CBCT_OK;
        }
    }
    cbct_plan *p = nullptr;
    cbct_geometry_desc g = r->g;
    g.angles = r->angles.empty() ? nullptr : r->angles.data();
    cbct_status st = cbct_plan_create(&s->ctx, &g, r->levels, 1, &p);
    if (st) return st;
    std::lock_guard<std::mutex> lk(s->pool_mu);
    auto it = s->plans.find(key);
    if (it != s->plans.end()) {  // another worker built it meanwhile
        cbct_plan_destroy(p);
        *out = it->second;
        return CBCT_OK;
    }
    s->plans.emplace(key, p);
    *out = p;
    return CBCT_OK;
}

void run_request(cbct_server *s, Request *r, hipStream_t stream) {
    if (s->simulated) {
        std::this_thread::sleep_for(std::chrono::duration<double>(r->sim_seconds));
        r->result = CBCT_OK;
        return;
    }
    cbct_plan *plan = nullptr;
    cbct_status st = get_plan(s, r, &plan);
    if (st) {
        r->result = st;
        r->err = cbct_last_error();
        return;
    }
    size_t ws_need = 0;
    r->p.iters = r->iters.data();
    st = cbct_reconstruct_workspace_size(plan, &r->p, &ws_need);
    if (!st && ws_need > r->ws_bytes)  // admission counted r->ws_bytes against the budget
        st = cbct_set_error(CBCT_ERR_INTERNAL, "server: workspace %zu bytes exceeds its admission estimate %zu",
                             ws_need, r->ws_bytes);
    Block ws{}, yb{};
    if (!st) {
        ws = block_get(s, ws_need);
        if (!ws.p) st = cbct_set_error(CBCT_ERR_OUT_OF_MEMORY, "server: workspace allocation of %zu bytes", ws.n);
    }
    const float *yd = r->y;
    const size_t ybytes = sizeof(float) * (size_t)r->g.n_views * r->g.nu * r->g.nv;
    if (!st && r->y_on_host) {
        yb = block_get(s, ybytes);
        if (!yb.p) st = cbct_set_error(CBCT_ERR_OUT_OF_MEMORY, "server: projection buffer of %zu bytes", ybytes);
        else if (hipMemcpyAsync(yb.p, r->y, ybytes, hipMemcpyHostToDevice, stream) != hipSuccess)
            st = cbct_set_error(CBCT_ERR_HIP, "server: projection upload failed");
        yd = (const float *)yb.p;
    }
    if (!st) st = cbct_reconstruct(plan, &r->p, yd, nullptr, r->d_out, ws.p, ws.n, (cbct_stream_t)stream, nullptr);
    if (!st && hipStreamSynchronize(stream) != hipSuccess) st = cbct_set_error(CBCT_ERR_HIP, "server: stream sync");
    if (st) r->err = cbct_last_error();
    pool_put(s, ws.p, ws.n);
    pool_put(s, yb.p, yb.n);
    r->result = st;
}

void worker_main(cbct_server *s) {
    hipStream_t stream = nullptr;
    if (!s->simulated) {
        hipSetDevice(s->ctx.device);
        hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    }
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] {
                return s->stop || (!s->queue.empty() && s->in_use + s->queue.front()->bytes <= s->budget);
            });
            if (s->queue.empty() || !(s->in_use + s->queue.front()->bytes <= s->budget)) {
                if (s->stop) break;
                continue;
            }
            r = s->queue.front();
            s->queue.pop_front();
            s->in_use += r->bytes;
            s->peak_in_use = std::max(s->peak_in_use, s->in_use);
            s->running++;
            s->peak_running = std::max(s->peak_running, s->running);
            r->t_start = clk::now();
        }
        s->cv_work.notify_all();  // the next head may fit as well
        run_request(s, r, stream);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->in_use -= r->bytes;
            s->running--;
            r->t_done = clk::now();
            r->done = true;
            s->completed++;
        }
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    if (stream) hipStreamDestroy(stream);
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
    if (!sim) s->ctx = *ctx;
    for (int w = 0; w < max_slots; w++) s->workers.emplace_back(worker_main, s);
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
    const int f = 1 << (p->levels - 1);
    if (g->nx % f || g->ny % f || g->nz % f || g->nu % f || g->nv % f)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit: dims not divisible by 2^(levels-1)");
    if (p->replay) return cbct_set_error(CBCT_ERR_INVALID_ARG, "server_submit: replay is a test-only solve option");
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
    r->ws_bytes = estimate_ws(*g, p->levels, r->iters, p->projector);
    const size_t tables = (size_t)p->levels * g->n_views * (g->nu * sizeof(ColParams) + sizeof(ViewParams));
    r->bytes = r->ws_bytes + tables + (y_on_host ? sizeof(float) * (size_t)g->n_views * g->nu * g->nv : 0);
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
    }
    s->cv_work.notify_all();
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
    if (in_use) *in_use = s->in_use;
    if (peak_in_use) *peak_in_use = s->peak_in_use;
    if (running) *running = s->running;
    if (peak_running) *peak_running = s->peak_running;
    if (queued) *queued = (int)s->queue.size();
    if (completed) *completed = s->completed;
    return CBCT_OK;
}

extern "C" void cbct_server_destroy(cbct_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    for (auto &kv : s->plans) cbct_plan_destroy(kv.second);
    if (!s->owned.empty()) {
        DeviceGuard dg(s->ctx.device);
        for (void *p : s->owned) hipFree(p);
    }
    delete s;
}
