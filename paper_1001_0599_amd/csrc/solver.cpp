// Reconstruction driver: Algorithm A1 of the paper (Section II.B) on every multigrid level
// (Section II.C.3), with Step 2 solved by gradient descent and the Armijo rule (Eq. 5).
//
// Per outer iteration, on the caller's stream (P, P^T: the trilinear pair or the Siddon pair):
//   P f - Y_l (residual epilogue of the projector)          -> r
//   g = f - kappa P^T r (epilogue of the adjoint gather)     Step 1, kappa = t * 2 N_vox / N_rays
//   u = g; ROF iterations: gradient pass, trial pass (4 step sizes), decision kernel, update
//   f = max(u, 0) fused with the copy into the projector's layout  Step 3
// The Armijo test and the stop test are evaluated on the device from FP64 sums; the host reads
// the 64-byte decision record once per ROF iteration to steer the loop.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>
#include <algorithm>

#include "cbct_internal.h"

namespace {

// Host-mapped pinned slot for the per-iteration decision record: the decision kernel writes it
// directly, so the host needs no copy command before reading it (a copy into pageable memory is
// staged through a runtime buffer on every ROF iteration).  One slot per host thread (the server
// runs solves on several threads), allocated on first use and never freed: a free from a
// thread-exit destructor could run after the HIP runtime has shut down.
// The same allocation holds the word of the gated loop's decisions, on its own cache line.
struct MappedSlot {
    RofControl *host = nullptr, *dev = nullptr;
    int *gword_host = nullptr, *gword_dev = nullptr;
};

MappedSlot mapped_ctl() {
    thread_local MappedSlot slot;
    thread_local bool tried = false;
    if (!tried) {
        tried = true;
        void *h = nullptr, *d = nullptr;
        if (hipHostMalloc(&h, 256, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
            hipHostGetDevicePointer(&d, h, 0) == hipSuccess) {
            slot.host = (RofControl *)h;
            slot.dev = (RofControl *)d;
            slot.gword_host = (int *)((char *)h + 128);
            slot.gword_dev = (int *)((char *)d + 128);
            *slot.gword_host = 0;
        } else {
            (void)hipGetLastError();  // fall back to copies; do not leave the error pending
        }
    }
    return slot;
}

// sequence numbers of the decision records of this host thread (never 0, the value the kernel
// writes into the record before its fields; they wrap within the gate word's 29 bits)
int next_seq() {
    thread_local int n = 0;
    n = (n + 1) & CBCT_GATE_SEQ_MASK;
    if (n == 0) n = 1;
    return n;
}

// is sequence number a at or after b (within half the ring)
bool seq_at_or_after(int a, int b) { return ((a - b) & CBCT_GATE_SEQ_MASK) < (CBCT_GATE_SEQ_MASK >> 1); }

// wait until the gate word carries a decision at or after `seq` and return it; after about 20 ms
// of polling, synchronise the stream (then every enqueued decision has written it)
cbct_status wait_gate(const int *word, int seq, hipStream_t s, int *out) {
    const volatile int *p = word;
    const auto t0 = std::chrono::steady_clock::now();
    for (int spin = 0;; spin++) {
        const int w = *p;
        if (seq_at_or_after(w >> 2, seq)) {
            *out = w;
            return CBCT_OK;
        }
        if ((spin & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) break;
    }
    CBCT_HIP(hipStreamSynchronize(s));
    const int w = *p;
    if (!seq_at_or_after(w >> 2, seq)) return cbct_set_error(CBCT_ERR_INTERNAL, "ROF gate: decision %d not seen", seq);
    *out = w;
    return CBCT_OK;
}

// wait until the host-mapped record carries `seq`: true when seen within the polling window
// (about 20 ms), false otherwise (the caller then synchronises the stream, after which the
// record is complete)
bool poll_seq(const RofControl *rec, int seq) {
    const volatile int *p = &rec->pad;
    const auto t0 = std::chrono::steady_clock::now();
    for (int spin = 0;; spin++) {
        if (*p == seq) {
            std::atomic_thread_fence(std::memory_order_acquire);
            return true;
        }
        if ((spin & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20))
            return false;
    }
}

std::mutex g_schur_mu;

// device-side records of cbct_tv_prox's Step 2 (one per ROF iteration, the default cap of 50 fits)
constexpr int TV_PROX_REC = 64;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Carver {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off = align256(off + count * sizeof(T));
        return p;
    }
};

using Bufs = SolveBufs;

size_t partial_count(const cbct_plan *p) {
    size_t m = (size_t)CBCT_RED_BLOCKS * (3 + 2 * CBCT_TRIALS);
    for (const auto &L : p->lv) m = std::max(m, (size_t)L.nviews * L.nu);
    return m;
}

// records of the device-side Step 2 (both the one-work-group loop and the gated chains), read
// back at each level's end: at most rof_max_iter per outer iteration of the level
int dev_rec_cap(const cbct_plan *, const cbct_solve_params *pr) {
    long cap = 0;
    for (int l = 0; l < pr->levels; l++) cap = std::max(cap, (long)std::max(pr->iters[l], 1) * pr->rof_max_iter);
    return (int)std::min<long>(cap, 1L << 24);
}

Bufs carve(const cbct_plan *p, int levels, int energy_slots, void *ws, int projector = 0, int rec_cap = 0,
          int replay_len = 0) {
    Carver c{(char *)ws};
    const Level &L0 = p->lv[0];
    Bufs b{};
    b.f = c.take<float>(L0.nvox());
    b.ft = c.take<float>(L0.nvox());
    b.g = c.take<float>(L0.nvox());
    b.u = c.take<float>(L0.nvox());
    b.d = c.take<float>(L0.nvox());
    b.r = c.take<float>(std::max(L0.nray(), L0.nvox()));
    // the adjoint's scratch: the trilinear pair's Z tables, or the Siddon pair's profile tables
    size_t zb = 0;
    for (int l = 0; l < levels; l++)
        zb = std::max(zb, projector == 1 ? cbct_adjoint_siddon_ws_bytes(p->lv[l]) : (size_t)p->lv[l].z_floats * 4);
    b.z = reinterpret_cast<float *>(c.take<char>(zb));
    for (int l = 0; l < 8; l++) b.ypyr[l] = nullptr;
    for (int l = 1; l < levels; l++)
        if (p->bin_detector) b.ypyr[l] = c.take<float>(p->lv[l].nray());
    b.part = c.take<double>(partial_count(p));
    b.sums = c.take<double>(64);
    b.eng = c.take<double>(2 * (size_t)std::max(energy_slots, 1));
    b.ctl = c.take<RofControl>(1);
    b.sst = c.take<RofLog>(1);
    b.gate = c.take<RofGate>(1);
    b.rec_cap = rec_cap;
    b.rec = c.take<RofRecord>(std::max(rec_cap, 1));
    b.replay = c.take<int>(2 * (size_t)std::max(replay_len, 1));
    b.bytes = c.off;
    return b;
}

cbct_status check_params(const cbct_plan *p, const cbct_solve_params *pr, const char *who) {
    if (!p || !pr) return cbct_set_error(CBCT_ERR_INVALID_ARG, "%s: NULL plan or params", who);
    if (pr->levels < 1 || pr->levels > p->levels)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "%s: params.levels %d not in [1, %d]", who, pr->levels, p->levels);
    if (!pr->iters) return cbct_set_error(CBCT_ERR_INVALID_ARG, "%s: params.iters is NULL", who);
    for (int l = 0; l < pr->levels; l++)
        if (pr->iters[l] < 0 || pr->iters[l] > 100000)
            return cbct_set_error(CBCT_ERR_INVALID_ARG, "%s: iters[%d] = %d out of range", who, l, pr->iters[l]);
    if (!(pr->lambda >= 0.0) || !(pr->tv_eps > 0.0) || !(pr->armijo_c > 0.0) || !(pr->backtrack > 0.0) ||
        !(pr->backtrack < 1.0) || !(pr->rof_tol >= 0.0) || pr->rof_max_iter < 0 || pr->rof_max_backtrack < 0)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "%s: invalid line-search or TV parameters", who);
    if (pr->replay_len < 0 || (pr->replay_len > 0 && !pr->replay))
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "%s: replay_len > 0 needs a replay array", who);
    if (!(pr->conv_tol >= 0.0)) return cbct_set_error(CBCT_ERR_INVALID_ARG, "%s: conv_tol < 0", who);
    if (pr->projector != 0 && pr->projector != 1)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "%s: projector %d is neither 0 nor 1", who, pr->projector);
    return CBCT_OK;
}

int energy_slots(const cbct_solve_params *pr) {
    int n = 0;
    for (int l = 0; l < pr->levels; l++) n += pr->iters[l] + 1;
    return n;
}

// Schur bound t = 1 / (kappa0 max(P 1) max(P^T 1)), cached per plan level and projector pair
cbct_status schur_step(cbct_plan *p, int level, int projector, const Bufs &b, hipStream_t s, double *t_out) {
    Level &L = p->lv[level];
    double &cached = projector == 1 ? L.schur_t_siddon : L.schur_t;
    {
        std::lock_guard<std::mutex> lk(g_schur_mu);
        if (cached > 0.0) {
            *t_out = cached;
            return CBCT_OK;
        }
    }
    cbct_status st;
    if ((st = cbct_launch_fill(b.ft, L.nvox(), 1.0f, s))) return st;
    st = projector == 1 ? cbct_launch_forward_siddon(L, b.ft, nullptr, b.r, nullptr, s)
                        : cbct_launch_forward(L, b.ft, nullptr, b.r, nullptr, s);
    if (st) return st;
    if ((st = cbct_launch_max(b.r, L.nray(), b.part, b.sums, s))) return st;
    if ((st = cbct_launch_fill(b.r, L.nray(), 1.0f, s))) return st;
    st = projector == 1 ? cbct_launch_adjoint_siddon(L, b.r, nullptr, 0.0f, b.u, b.z, s)
                        : cbct_launch_adjoint(L, b.r, nullptr, 0.0f, b.u, b.z, s);
    if (st) return st;
    if ((st = cbct_launch_max(b.u, L.nvox(), b.part, b.sums + 1, s))) return st;
    double mx[2];
    CBCT_HIP(hipMemcpyAsync(mx, b.sums, sizeof(mx), hipMemcpyDeviceToHost, s));
    CBCT_HIP(hipStreamSynchronize(s));
    const double kappa0 = 2.0 * (double)L.nvox() / (double)L.nray();
    const double lip = kappa0 * mx[0] * mx[1];
    if (!(lip > 0.0) || !std::isfinite(lip))
        return cbct_set_error(CBCT_ERR_NONFINITE, "level %d: Schur bound %g is not positive and finite", level, lip);
    std::lock_guard<std::mutex> lk(g_schur_mu);
    cached = 1.0 / lip;
    *t_out = cached;
    return CBCT_OK;
}

struct TraceSink {
    cbct_solve_stats *st;
    void push(int level, int outer, int inner, int m, const RofControl &c) {
        if (!st) return;
        int k = st->trace_len;
        if (st->trace && k < st->trace_cap) {
            st->trace[4 * k + 0] = level;
            st->trace[4 * k + 1] = outer;
            st->trace[4 * k + 2] = inner;
            st->trace[4 * k + 3] = m;
            if (st->rof_e) {
                st->rof_e[3 * k + 0] = c.e0;
                st->rof_e[3 * k + 1] = c.e_trial;
                st->rof_e[3 * k + 2] = c.G;
            }
        }
        st->trace_len = k + 1;
    }
};

// Reads back a level's device-side Step 2 log: its state (replay records consumed, a
// non-finite energy) and, for the caller's statistics, its per-iteration records in order.
cbct_status flush_step2_log(const Bufs &b, hipStream_t s, TraceSink &sink, int *replay_pos) {
    RofLog st;
    CBCT_HIP(hipMemcpyAsync(&st, b.sst, sizeof(st), hipMemcpyDeviceToHost, s));
    CBCT_HIP(hipStreamSynchronize(s));
    if (replay_pos) *replay_pos = st.replay_pos;
    const int n = std::min(st.n_rec, b.rec_cap);
    if (sink.st && n > 0) {
        std::vector<RofRecord> rec(n);
        CBCT_HIP(hipMemcpyAsync(rec.data(), b.rec, sizeof(RofRecord) * n, hipMemcpyDeviceToHost, s));
        CBCT_HIP(hipStreamSynchronize(s));
        for (const RofRecord &r : rec) {
            RofControl c{};
            c.e0 = r.e0;
            c.e_trial = r.e_trial;
            c.G = r.G;
            sink.push(r.level, r.outer, r.inner, r.m, c);
        }
    }
    if (st.status) return cbct_set_error(CBCT_ERR_NONFINITE, "ROF energy is not finite (device-side Step 2)");
    return CBCT_OK;
}

// Step 2 driven from the host (Step 2 alone with a replay, or with more ROF iterations than its
// record buffer holds): u = ROF(g) from u = g, one read of the device's decision per backtracking
// window.  `replay_pos` walks params.replay.
cbct_status rof_loop(const Level &L, const cbct_solve_params *pr, double t, const Bufs &b, hipStream_t s,
                     TraceSink &sink, int level, int outer, int *replay_pos) {
    cbct_status st;
    CBCT_HIP(hipMemcpyAsync(b.u, b.g, sizeof(float) * L.nvox(), hipMemcpyDeviceToDevice, s));
    for (int it = 0; it < pr->rof_max_iter; it++) {
        int forced = -2;      // free running
        int forced_end = -1;  // replayed: 1 when this record ends Step 2
        if (pr->replay && *replay_pos < pr->replay_len) {
            forced = pr->replay[2 * *replay_pos];
            forced_end = pr->replay[2 * *replay_pos + 1] != 0 ? 1 : 0;
            (*replay_pos)++;
        }
        if ((st = cbct_launch_tv_grad(L, pr->tv_eps, b.u, b.g, b.d, pr->lambda, t, b.part, b.sums, s))) return st;
        RofControl c{};
        if (forced == -1) {
            // replayed decision: the search found no admissible step
            double sums[3];
            CBCT_HIP(hipMemcpyAsync(sums, b.sums, sizeof(sums), hipMemcpyDeviceToHost, s));
            CBCT_HIP(hipStreamSynchronize(s));
            const double inv_n = 1.0 / (double)L.nvox();
            c.e0 = pr->lambda * sums[0] * inv_n + sums[1] * inv_n / (2.0 * t);
            c.G = sums[2] * inv_n;
            c.accepted = -1;
            sink.push(level, outer, it, -1, c);
            break;
        }
        // the first window tries the full step only (it is accepted almost always); later
        // windows try CBCT_TRIALS step sizes per pass
        int m0 = 0;
        for (;;) {
            const int M = (m0 == 0) ? 1 : CBCT_TRIALS;
            if ((st = cbct_launch_tv_trial(L, pr->tv_eps, b.u, b.d, b.g, t, pr->backtrack, m0, M, b.part, b.sums + 3,
                                           s)))
                return st;
            const MappedSlot ms = mapped_ctl();
            const int seq = next_seq();
            if ((st = cbct_launch_rof_decide(b.sums, m0, M, forced >= 0 ? forced : -1, L.nvox(), pr->lambda, t,
                                             pr->armijo_c, pr->backtrack, pr->rof_max_backtrack, b.ctl, ms.dev, seq,
                                             s)))
                return st;
            if (ms.host) {
                // the record is complete once its sequence number shows: poll it for a while (the
                // kernel writes it before the stream reports completion), then block on the stream
                if (!poll_seq(ms.host, seq)) CBCT_HIP(hipStreamSynchronize(s));
                std::memcpy(&c, ms.host, sizeof(c));
            } else {
                CBCT_HIP(hipMemcpyAsync(&c, b.ctl, sizeof(c), hipMemcpyDeviceToHost, s));
                CBCT_HIP(hipStreamSynchronize(s));
            }
            if (c.accepted == 0 && c.next_m0 > m0) {
                m0 = c.next_m0;
                continue;
            }
            break;
        }
        if (!std::isfinite(c.e0) || !std::isfinite(c.G))
            return cbct_set_error(CBCT_ERR_NONFINITE, "ROF energy is not finite (level %d, outer %d)", level, outer);
        sink.push(level, outer, it, c.accepted == 1 ? c.m : -1, c);
        if (c.accepted != 1) break;  // Eq. 5 held for no step: keep u
        const bool own_stop = c.e0 == 0.0 || c.G == 0.0 || std::fabs(c.e_trial - c.e0) / c.e0 < pr->rof_tol;
        const bool stop = (forced_end >= 0 ? forced_end == 1 : own_stop) || it + 1 == pr->rof_max_iter;
        if ((st = cbct_launch_axpy_step(b.u, b.d, b.ctl, L.nvox(), s))) return st;
        if (stop) break;
    }
    return CBCT_OK;
}

// Step 2 of a larger level as flag-gated launch chains: u = ROF(g) from u already holding g.  The
// steps go out AHEAD at a time in front of the decisions; the host waits for one decision word
// per step (not per pass), so the device runs the ROF iterations and backtracking windows back to
// back, and the host stops enqueueing when a decision ends the loop (a step enqueued past the end
// does nothing).  `first`: the level's first loop (resets the records and replay position).
// With `apply_pending` an accepted step that ends the loop is applied to u here; otherwise it is
// left to the caller's Step 3 (the clamp applies it when the last decision accepted a step).
cbct_status rof_loop_gated(const Level &L, const cbct_solve_params *pr, double t, const Bufs &b, hipStream_t s,
                           int level, int outer, bool first, int replay_pos, bool records, bool apply_pending) {
    constexpr int AHEAD = 2;
    cbct_status st;
    const MappedSlot ms = mapped_ctl();
    RofStepArgs a{};
    a.eps = pr->tv_eps;
    a.lambda = pr->lambda;
    a.t = t;
    a.c_armijo = pr->armijo_c;
    a.alpha = pr->backtrack;
    a.tol = pr->rof_tol;
    a.max_iter = pr->rof_max_iter;
    a.max_bt = pr->rof_max_backtrack;
    a.u = b.u;
    a.g = b.g;
    a.d = b.d;
    a.part = b.part;
    a.sums = b.sums;
    a.ctl = b.ctl;
    a.gate = b.gate;
    a.st = b.sst;
    a.replay = pr->replay ? b.replay : nullptr;
    a.replay_len = pr->replay ? pr->replay_len : 0;
    a.rec = records ? b.rec : nullptr;
    a.rec_cap = b.rec_cap;
    a.level = level;
    a.outer = outer;
    a.mirror = ms.gword_dev;
    // steps one loop can take: per ROF iteration the first window and at most
    // ceil(max_bt / CBCT_TRIALS) more
    const long max_steps = (long)pr->rof_max_iter * (2 + pr->rof_max_backtrack / CBCT_TRIALS);
    std::vector<int> seqs;
    long known = 0;  // steps whose decisions left the loop running
    for (;;) {
        while ((long)seqs.size() < max_steps && (long)seqs.size() < known + AHEAD) {
            a.seq = next_seq();
            a.first = seqs.empty() ? 1 : 0;
            a.init_state = (a.first && first) ? 1 : 0;
            a.replay_pos = replay_pos;
            seqs.push_back(a.seq);
            if ((st = cbct_launch_rof_step_gated(L, a, s))) return st;
        }
        if (known >= (long)seqs.size()) break;  // every step a loop can take has run
        int w;
        if (ms.gword_host) {
            if ((st = wait_gate(ms.gword_host, seqs[known], s, &w))) return st;
        } else {
            // no host-mapped word: read the state after the enqueued steps
            RofGate gs;
            RofLog ss;
            CBCT_HIP(hipMemcpyAsync(&gs, b.gate, sizeof(gs), hipMemcpyDeviceToHost, s));
            CBCT_HIP(hipMemcpyAsync(&ss, b.sst, sizeof(ss), hipMemcpyDeviceToHost, s));
            CBCT_HIP(hipStreamSynchronize(s));
            w = cbct_gate_word(seqs.back(), ss.status ? 1 : 0, gs.run);
        }
        if (w & 2) return cbct_set_error(CBCT_ERR_NONFINITE, "ROF energy is not finite (level %d, outer %d)", level, outer);
        if (!(w & 1)) break;  // the loop has ended
        // the word names the latest decision taken: every step up to it left the loop running
        long idx = known;
        while (idx + 1 < (long)seqs.size() && seqs[idx] != (w >> 2)) idx++;
        known = idx + 1;
    }
    if (apply_pending && (st = cbct_launch_axpy_pending(b.u, b.d, b.ctl, b.gate, L.nvox(), s))) return st;
    return CBCT_OK;
}

}  // namespace

SolveBufs cbct_solve_carve(const cbct_plan *p, const cbct_solve_params *pr, void *ws) {
    return carve(p, pr->levels, energy_slots(pr), ws, pr->projector, dev_rec_cap(p, pr),
                 pr->replay ? pr->replay_len : 0);
}

cbct_status cbct_solve_schur(cbct_plan *p, int level, int projector, const SolveBufs &b, hipStream_t s, double *t) {
    return schur_step(p, level, projector, b, s, t);
}

extern "C" void cbct_solve_params_default(cbct_solve_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->lambda = 0.05;
    p->levels = 1;
    p->step = 0.0;
    p->tv_eps = 1e-5;
    p->armijo_c = 0.01;
    p->backtrack = 0.6;
    p->rof_tol = 1e-3;
    p->rof_max_iter = 50;
    p->rof_max_backtrack = 30;
}

extern "C" cbct_status cbct_reconstruct_workspace_size(const cbct_plan *p, const cbct_solve_params *pr,
                                                       size_t *bytes) {
    cbct_status st = check_params(p, pr, "reconstruct_workspace_size");
    if (st) return st;
    if (!bytes) return cbct_set_error(CBCT_ERR_INVALID_ARG, "reconstruct_workspace_size: NULL out");
    *bytes = carve(p, pr->levels, energy_slots(pr), nullptr, pr->projector, dev_rec_cap(p, pr),
                   pr->replay ? pr->replay_len : 0).bytes;
    return CBCT_OK;
}

extern "C" cbct_status cbct_reconstruct(cbct_plan *p, const cbct_solve_params *pr, const float *d_y,
                                        const float *d_init, float *d_out, void *d_ws, size_t ws_bytes,
                                        cbct_stream_t stream, cbct_solve_stats *stats) {
    const auto t_start = std::chrono::steady_clock::now();
    cbct_status st = check_params(p, pr, "reconstruct");
    if (st) return st;
    if (!d_y || !d_out || !d_ws) return cbct_set_error(CBCT_ERR_INVALID_ARG, "reconstruct: NULL pointer");
    DeviceGuard dg(p->device);
    const int levels = pr->levels;
    const int nslots = energy_slots(pr);
    const int proj = pr->projector;
    Bufs b = carve(p, levels, nslots, d_ws, proj, dev_rec_cap(p, pr), pr->replay ? pr->replay_len : 0);
    if (ws_bytes < b.bytes)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "reconstruct: workspace %zu < %zu bytes", ws_bytes, b.bytes);
    if (((uintptr_t)d_ws & 255) != 0)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "reconstruct: workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    if (stats) {
        stats->trace_len = 0;
        stats->energy_len = 0;
        stats->replay_used = 0;
        for (int l = 0; l < 8; l++) stats->t_used[l] = 0.0;
    }
    TraceSink sink{stats};
    if (pr->replay && pr->replay_len > 0)
        CBCT_HIP(hipMemcpyAsync(b.replay, pr->replay, sizeof(int) * 2 * (size_t)pr->replay_len, hipMemcpyHostToDevice,
                                s));
    const bool want_energy = stats && stats->energy;
    const bool conv = pr->conv_tol > 0.0;  // the stop rule needs E(f_k) on the host every iteration
    std::vector<int> slots_of_level(levels, 0);
    int replay_pos = 0;
    int eslot = 0;
    const Level &L0 = p->lv[0];

    // coarsest start: 0, or d_init restricted level by level
    {
        const Level &Lc = p->lv[levels - 1];
        if (d_init) {
            const float *src = d_init;
            float *bufs[2] = {b.g, b.u};
            for (int l = 1; l < levels; l++) {
                float *dst = (l == levels - 1) ? b.f : bufs[l & 1];
                if ((st = cbct_launch_restrict(p->lv[l], src, dst, s))) return st;
                src = dst;
            }
            if (levels == 1) CBCT_HIP(hipMemcpyAsync(b.f, d_init, sizeof(float) * L0.nvox(), hipMemcpyDeviceToDevice, s));
        } else {
            if ((st = cbct_launch_fill(b.f, Lc.nvox(), 0.0f, s))) return st;
        }
    }
    for (int l = levels - 1; l >= 0; l--) {
        const Level &L = p->lv[l];
        if (l < levels - 1) {
            if ((st = cbct_launch_prolong(p->lv[l + 1], b.f, b.u, s))) return st;
            std::swap(b.f, b.u);
        }
        const float *Yl = d_y;
        if (l > 0 && p->bin_detector) {
            if ((st = cbct_launch_bin(L0, 1 << l, d_y, b.ypyr[l], s))) return st;
            Yl = b.ypyr[l];
        }
        double t = pr->step;
        if (!(t > 0.0))
            if ((st = schur_step(p, l, proj, b, s, &t))) return st;
        if (stats) stats->t_used[l] = t;
        const float kappa = (float)(t * 2.0 * (double)L.nvox() / (double)L.nray());
        if ((st = cbct_launch_to_columns(L, b.f, b.ft, s))) return st;
        // Step 2 runs on the device: small levels in one work-group, larger ones as gated launch
        // chains; the records and the replay position come back once, at the level's end
        const bool small = L.nvox() <= CBCT_SMALL_ROF_VOX && b.rec_cap > 0;
        bool dev_ran = false;
        double e_prev = 0.0;
        for (int k = 0; k <= pr->iters[l]; k++) {
            const bool last = (k == pr->iters[l]);
            if (last && !want_energy) break;
            // residual r = P f - Y_l and its sum of squares (the trilinear pair hands its exact
            // adjoint the ray-weighted residual)
            const bool eq6 = pr->step1_eq6 != 0;
            st = proj == 1 ? cbct_launch_forward_siddon(L, b.ft, Yl, b.r, b.part, s)
                           : cbct_launch_forward(L, b.ft, Yl, b.r, b.part, s, !eq6);
            if (st) return st;
            if (want_energy || conv) {
                if ((st = cbct_launch_sum_rows(b.part, L.nviews * L.nu, 1, b.eng + 2 * eslot, s))) return st;
                if ((st = cbct_launch_tv_energy(L, pr->tv_eps, b.f, b.part, b.eng + 2 * eslot + 1, s))) return st;
                eslot++;
                slots_of_level[l]++;
            }
            if (conv) {
                // "until convergence": f_k is final once the energy stalls
                double e2[2];
                CBCT_HIP(hipMemcpyAsync(e2, b.eng + 2 * (eslot - 1), sizeof(e2), hipMemcpyDeviceToHost, s));
                CBCT_HIP(hipStreamSynchronize(s));
                const double Ek = e2[0] / (double)L.nray() + pr->lambda * e2[1] / (double)L.nvox();
                if (!std::isfinite(Ek))
                    return cbct_set_error(CBCT_ERR_NONFINITE, "energy is not finite (level %d, outer %d)", l, k);
                if (k >= 1 && std::fabs(Ek - e_prev) <= pr->conv_tol * e_prev) break;
                e_prev = Ek;
            }
            if (last) break;
            // Step 1: g = f - kappa P^T r, or with the Eq. 6 backprojector in place of P^T
            // (each writes the ROF start u = g as well)
            if (eq6)
                st = cbct_launch_backproject_eq6(L, b.r, b.f, kappa, b.g, s, b.u);
            else if (proj == 1)
                st = cbct_launch_adjoint_siddon(L, b.r, b.f, kappa, b.g, b.z, s, b.u);
            else
                st = cbct_launch_adjoint(L, b.r, b.f, kappa, b.g, b.z, s, true, b.u);
            if (st) return st;
            // Step 2
            bool pending = false;
            if (small) {
                st = cbct_launch_rof_small(L, pr->tv_eps, b.u, b.g, b.d, pr->lambda, t, pr->armijo_c, pr->backtrack,
                                           pr->rof_tol, pr->rof_max_iter, pr->rof_max_backtrack,
                                           pr->replay ? b.replay : nullptr, pr->replay ? pr->replay_len : 0,
                                           replay_pos, b.sst, stats ? b.rec : nullptr, b.rec_cap, l, k, !dev_ran, s);
                if (st) return st;
                dev_ran = true;
            } else if (pr->rof_max_iter > 0) {
                if ((st = rof_loop_gated(L, pr, t, b, s, l, k, !dev_ran, replay_pos, stats != nullptr, false)))
                    return st;
                dev_ran = true;
                pending = true;  // the clamp applies the last decision's step if it accepted one
            }
            // Step 3 (with the last ROF update when it is pending)
            if ((st = cbct_launch_clamp_columns(L, b.u, b.f, b.ft, s, pending ? b.d : nullptr,
                                                pending ? b.ctl : nullptr)))
                return st;
        }
        if (dev_ran && (st = flush_step2_log(b, s, sink, &replay_pos))) return st;
    }
    CBCT_HIP(hipMemcpyAsync(d_out, b.f, sizeof(float) * L0.nvox(), hipMemcpyDeviceToDevice, s));
    if (stats) {
        stats->replay_used = replay_pos;
        if (want_energy) {
            std::vector<double> e(2 * (size_t)eslot);
            if (eslot) CBCT_HIP(hipMemcpyAsync(e.data(), b.eng, sizeof(double) * e.size(), hipMemcpyDeviceToHost, s));
            CBCT_HIP(hipStreamSynchronize(s));
            int idx = 0;
            for (int l = levels - 1; l >= 0; l--) {
                const Level &L = p->lv[l];
                for (int k = 0; k < slots_of_level[l]; k++, idx++) {
                    const double E = e[2 * idx] / (double)L.nray() + pr->lambda * e[2 * idx + 1] / (double)L.nvox();
                    if (stats->energy_len < stats->energy_cap) stats->energy[stats->energy_len] = E;
                    stats->energy_len++;
                }
            }
        }
        CBCT_HIP(hipStreamSynchronize(s));
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    }
    return CBCT_OK;
}

extern "C" cbct_status cbct_tv_prox_workspace_size(const cbct_plan *p, int level, size_t *bytes) {
    if (!p || !bytes || level < 0 || level >= p->levels)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "tv_prox_workspace_size: bad arguments");
    cbct_solve_params pr;
    cbct_solve_params_default(&pr);
    int it = 0;
    pr.iters = &it;
    *bytes = carve(p, 1, 1, nullptr, 0, TV_PROX_REC).bytes;
    return CBCT_OK;
}

extern "C" cbct_status cbct_tv_prox(cbct_plan *p, int level, const cbct_solve_params *pr, const float *d_g,
                                    float *d_u, void *d_ws, size_t ws_bytes, cbct_stream_t stream,
                                    cbct_solve_stats *stats) {
    if (!p || !pr || !d_g || !d_u || !d_ws || level < 0 || level >= p->levels)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "tv_prox: bad arguments");
    if (!(pr->step > 0.0)) return cbct_set_error(CBCT_ERR_INVALID_ARG, "tv_prox: params.step (t) must be > 0");
    DeviceGuard dg(p->device);
    Bufs b = carve(p, 1, 1, d_ws, 0, TV_PROX_REC);
    if (ws_bytes < b.bytes) return cbct_set_error(CBCT_ERR_INVALID_ARG, "tv_prox: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const Level &L = p->lv[level];
    if (stats) stats->trace_len = 0;
    TraceSink sink{stats};
    int pos = 0;
    CBCT_HIP(hipMemcpyAsync(b.g, d_g, sizeof(float) * L.nvox(), hipMemcpyDeviceToDevice, s));
    cbct_status st;
    if (L.nvox() <= CBCT_SMALL_ROF_VOX && pr->rof_max_iter <= b.rec_cap && !pr->replay) {
        // the whole loop in one work-group on the device, read back once
        CBCT_HIP(hipMemcpyAsync(b.u, b.g, sizeof(float) * L.nvox(), hipMemcpyDeviceToDevice, s));
        if ((st = cbct_launch_rof_small(L, pr->tv_eps, b.u, b.g, b.d, pr->lambda, pr->step, pr->armijo_c, pr->backtrack,
                                        pr->rof_tol, pr->rof_max_iter, pr->rof_max_backtrack, nullptr, 0, 0, b.sst,
                                        b.rec, b.rec_cap, level, 0, true, s)))
            return st;
        if ((st = flush_step2_log(b, s, sink, &pos))) return st;
    } else if (!pr->replay && pr->rof_max_iter > 0 && (!stats || pr->rof_max_iter <= b.rec_cap)) {
        // gated launch chains, records read back once
        CBCT_HIP(hipMemcpyAsync(b.u, b.g, sizeof(float) * L.nvox(), hipMemcpyDeviceToDevice, s));
        if ((st = rof_loop_gated(L, pr, pr->step, b, s, level, 0, true, 0, stats != nullptr, true))) return st;
        if ((st = flush_step2_log(b, s, sink, &pos))) return st;
    } else if ((st = rof_loop(L, pr, pr->step, b, s, sink, level, 0, &pos))) {
        return st;
    }
    CBCT_HIP(hipMemcpyAsync(d_u, b.u, sizeof(float) * L.nvox(), hipMemcpyDeviceToDevice, s));
    if (stats) stats->replay_used = pos;
    return CBCT_OK;
}

extern "C" cbct_status cbct_tv_energy_grad_workspace_size(const cbct_plan *p, size_t *bytes) {
    if (!p || !bytes) return cbct_set_error(CBCT_ERR_INVALID_ARG, "tv_energy_grad_workspace_size: NULL argument");
    *bytes = sizeof(double) * (CBCT_RED_BLOCKS * 3 + 8);
    return CBCT_OK;
}

extern "C" cbct_status cbct_tv_energy_grad(cbct_plan *p, int level, double tv_eps, const float *d_f, float *d_grad,
                                           double *h_sum, void *d_ws, size_t ws_bytes, cbct_stream_t stream) {
    if (!p || !d_f || !d_ws || level < 0 || level >= p->levels || !(tv_eps > 0.0))
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "tv_energy_grad: bad arguments");
    const size_t need = sizeof(double) * (CBCT_RED_BLOCKS * 3 + 8);
    if (ws_bytes < need) return cbct_set_error(CBCT_ERR_INVALID_ARG, "tv_energy_grad: workspace < %zu bytes", need);
    const Level &L = p->lv[level];
    hipStream_t s = (hipStream_t)stream;
    DeviceGuard dg(p->device);
    double *part = (double *)d_ws, *sums = part + CBCT_RED_BLOCKS * 3;
    cbct_status st;
    if (d_grad) st = cbct_launch_tv_grad(L, tv_eps, d_f, nullptr, d_grad, 0.0, 1.0, part, sums, s);
    else st = cbct_launch_tv_energy(L, tv_eps, d_f, part, sums, s);
    if (st) return st;
    if (h_sum) {
        CBCT_HIP(hipMemcpyAsync(h_sum, sums, sizeof(double), hipMemcpyDeviceToHost, s));
        CBCT_HIP(hipStreamSynchronize(s));
    }
    return CBCT_OK;
}

extern "C" cbct_status cbct_tv_energy_grad_noalloc(cbct_plan *p, int level, double tv_eps, const float *d_f,
                                                   float *d_grad, double *h_sum, cbct_stream_t stream) {
    if (!p || !d_f || level < 0 || level >= p->levels || !(tv_eps > 0.0))
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "tv_energy_grad_noalloc: bad arguments");
    const Level &L = p->lv[level];
    // the same partial-sum layout as cbct_tv_energy_grad, in the device's scratch array
    const size_t need = sizeof(double) * ((size_t)CBCT_RED_BLOCKS * 3 + 8);
    if (need > CBCT_NOALLOC_SCRATCH_BYTES || (size_t)cbct_reduce_blocks(L) > (size_t)CBCT_RED_BLOCKS)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "tv_energy_grad_noalloc: needs %zu bytes of scratch, the maximum is %zu",
                              need, CBCT_NOALLOC_SCRATCH_BYTES);
    double *part = (double *)cbct_noalloc_scratch(p->device);
    if (!part)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "tv_energy_grad_noalloc: no context was created for device %d",
                              p->device);
    double *sums = part + CBCT_RED_BLOCKS * 3;
    hipStream_t s = (hipStream_t)stream;
    DeviceGuard dg(p->device);
    // every partial the final sum reads is written by this call's gradient (or energy) pass:
    // nothing in the scratch needs clearing first
    cbct_status st;
    if (d_grad) st = cbct_launch_tv_grad(L, tv_eps, d_f, nullptr, d_grad, 0.0, 1.0, part, sums, s);
    else st = cbct_launch_tv_energy(L, tv_eps, d_f, part, sums, s);
    if (st) return st;
    if (h_sum) {
        CBCT_HIP(hipMemcpyAsync(h_sum, sums, sizeof(double), hipMemcpyDeviceToHost, s));
        CBCT_HIP(hipStreamSynchronize(s));
    }
    return CBCT_OK;
}

extern "C" cbct_status cbct_prolong(const cbct_plan *p, int coarse_level, const float *d_c, float *d_f,
                                    cbct_stream_t stream) {
    if (!p || !d_c || !d_f || coarse_level < 1 || coarse_level >= p->levels)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "prolong: bad arguments");
    DeviceGuard dg(p->device);
    return cbct_launch_prolong(p->lv[coarse_level], d_c, d_f, (hipStream_t)stream);
}

extern "C" cbct_status cbct_restrict(const cbct_plan *p, int fine_level, const float *d_f, float *d_c,
                                     cbct_stream_t stream) {
    if (!p || !d_c || !d_f || fine_level < 0 || fine_level + 1 >= p->levels)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "restrict: bad arguments");
    DeviceGuard dg(p->device);
    return cbct_launch_restrict(p->lv[fine_level + 1], d_f, d_c, (hipStream_t)stream);
}

extern "C" cbct_status cbct_bin_detector(const cbct_plan *p, int level, const float *d_y0, float *d_yl,
                                         cbct_stream_t stream) {
    if (!p || !d_y0 || !d_yl || level < 1 || level >= p->levels || !p->bin_detector)
        return cbct_set_error(CBCT_ERR_INVALID_ARG, "bin_detector: bad arguments (level >= 1, plan with binning)");
    DeviceGuard dg(p->device);
    return cbct_launch_bin(p->lv[0], 1 << level, d_y0, d_yl, (hipStream_t)stream);
}
