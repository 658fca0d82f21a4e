"""Benchmark of the FBS-TV cone-beam reconstruction hot path on one MI355X.

A step is one full reconstruction of the 512x512x64-voxel (0.9x0.9x2.5 mm), 40-view,
512x384-detector workload: 2 multigrid levels x 20 outer iterations of Algorithm A1 (P with
residual, P^T with the Step-1 update, the ROF prox with Armijo line search, the non-negativity
clamp, multigrid transfers), lambda = 0.05, Schur-bound step (computed once per plan, in
warm-up).  Inputs (projections) are resident in HBM before the timed region.

Prints ONE JSON line.  `value` is the whole-job P/P^T throughput: the voxel*views of every
P and P^T application in a reconstruction divided by the reconstruction's wall time.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# HBM traffic and L2 hit rate of the P^T operator per launch, from hardware counters (FETCH_SIZE
# and WRITE_SIZE, each scaled by what the counter reads for a plain copy of known size; TCC_HIT and
# TCC_MISS).  The record names the sources it was measured on; it is reported only while they are
# unchanged.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "adjoint_traffic_512x512x64_40views.txt")
TRAFFIC_SOURCES = ["backproject.hip", "adj_profiles.h", "geometry_tables.h", "plan.cpp"]


def sources_digest(names):
    import hashlib
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1001_0599_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """(HBM bytes per launch, L2 hit rate) of P^T from the committed counter record, or
    (None, None) if it is missing or stale."""
    try:
        with open(TRAFFIC_RECORD) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(" "))
    except OSError:
        return None, None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("sources_sha256") != sources_digest(TRAFFIC_SOURCES):
        return None, None
    try:
        return float(kv["hbm_bytes_per_launch"]), float(kv.get("l2_hit_rate", "nan"))
    except (KeyError, ValueError):
        return None, None


def host_cpu():
    """The host's CPU model (from /proc/cpuinfo) and the logical CPUs the OS reports."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def cpu_baseline(g, iters, lam):
    """The FP64 oracle on the host cores, on bounded samples of the workload:
    - all threads: P and P^T of 12 of the 40 views (every ray of those views, the full volume),
      scaled to voxel*views/s (`value`);
    - one thread: P and P^T of 2 of the 40 views, the same scaling (`value_1thread`);
    - the oracle's whole reconstruction ([20, 20] outer iterations, both levels), extrapolated
      from timed pieces on all threads: per level, P and P^T of the level (the fine level from
      the 12-view sample scaled to 40 views, the coarse level over all 40 views) plus one ROF
      solve (Step 2) of the level's volume, times the level's outer iterations."""
    import dataclasses

    import numpy as np

    import cbct_synth as S
    import oracle

    def sample(gg, nv):
        return dataclasses.replace(gg, n_views=nv, angles=tuple(2 * np.pi * (q * gg.n_views // nv) / gg.n_views
                                                               for q in range(nv)))

    def time_pair(gg):
        x = S.random_volume(gg, 1)
        y = S.random_projections(gg, 2)
        t0 = time.perf_counter()
        oracle.forward(gg, x)
        t1 = time.perf_counter()
        oracle.adjoint(gg, y)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    oracle.lib()
    threads = oracle.get_threads()
    nv = 12
    tp, ta = time_pair(sample(g, nv))
    vv = g.n_vox * nv
    res = {"value": 2 * vv / (tp + ta), "unit": "voxel·views/s", "cores": threads, "kind": "oracle",
           "sample": "P and P^T of 12 of the 40 views (all 196608 rays each, full 512x512x64 volume), FP64; "
                     "P %.2f s, P^T %.2f s" % (tp, ta)}
    # one thread, 2 views
    oracle.set_threads(1)
    try:
        tp1, ta1 = time_pair(sample(g, 2))
    finally:
        oracle.set_threads(threads)
    res["value_1thread"] = 2 * g.n_vox * 2 / (tp1 + ta1)
    res["sample_1thread"] = "P and P^T of 2 of the 40 views on 1 thread: P %.2f s, P^T %.2f s" % (tp1, ta1)
    # extrapolated oracle reconstruction
    per_level = []
    for lvl, it in enumerate(iters):
        gl = S.level_geometry(g, lvl)
        if lvl == 0:
            pt = (tp + ta) * g.n_views / nv
        else:
            a, b = time_pair(gl)
            pt = a + b
        f = np.clip(S.random_volume(gl, 3) * 0.02, 0.0, None)
        t0 = time.perf_counter()
        r = oracle.rof(gl, f, lam, 1e-3)
        rof_s = time.perf_counter() - t0
        per_level.append((lvl, it, pt, rof_s, len(r.trace)))
    total = sum(it * (pt + rof_s) for _, it, pt, rof_s, _ in per_level)
    res["recon_s_extrapolated"] = total
    res["recon_extrapolation"] = (
        "EXTRAPOLATED, not run: sum over levels of iters x (P + P^T + one Step-2 solve), each timed once on %d "
        "threads: " % threads + "; ".join("level %d: %d x (%.2f s + %.2f s for %d ROF iterations)"
                                          % (lvl, it, pt, rof_s, n) for lvl, it, pt, rof_s, n in per_level))
    return res


def plain_replay(arrivals, reqs, make):
    """The plain one-at-a-time solver on the same GPU: requests in arrival order, each solved by
    cbct_reconstruct (plans cached per geometry, like the server's) as soon as it has arrived and
    the previous one is done.  Returns latencies (completion - arrival) and the span."""
    import numpy as np
    import torch

    from paper_1001_0599_amd.ops import Plan

    plans = {}
    t0 = time.perf_counter()
    done = np.zeros(len(arrivals))
    for r, ta in enumerate(arrivals):
        dt = ta - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        kw = make(r)
        g = kw["geom"]
        key = (g.nx, g.ny, g.nz, g.n_views, g.nu, g.nv)
        if key not in plans:
            plans[key] = Plan(g)
        plans[key].reconstruct(kw["y"], lam=kw["lam"], iters=kw["iters"], out=kw["out"])
        torch.cuda.synchronize()
        done[r] = time.perf_counter() - t0
    lat = done - np.asarray(arrivals)
    return lat, float(done.max() - arrivals[0])


def serving_run(n_requests):
    """The serving workload: n requests with Poisson arrivals (4/s), volumes uniform over
    {64^3, 128^3, 256x256x96} at 2 mm, 20-120 views, detector 2Nx x 2Nz at 1.5 mm, 30 iterations,
    200 GB budget; the continuous-admission server (8 slots, batched engines) against the plain
    solver one request at a time on the same arrivals, then both with all requests submitted at
    once (saturation).  Served results are checked bitwise against the plain ones."""
    import numpy as np
    import torch

    import cbct_synth as S
    from paper_1001_0599_amd.serving import Server, replay, summarize

    cfg = S.CONFIGS["serving_mix"]
    reqs = S.serving_requests(n_requests)
    log("serving: synthesising %d requests on the GPU" % n_requests)
    ys, outs, ref = [], [], []
    for r in reqs:
        g = r["geometry"]
        ph = S.make_phantom(g, r["phantom_seed"])
        p = S.analytic_projections_torch(g, ph, "cuda")
        ys.append(S.poisson_log_torch(p, cfg["I0"], r["noise_seed"]).float().contiguous())
        outs.append(torch.empty(g.vol_shape, device="cuda"))
        ref.append(torch.empty(g.vol_shape, device="cuda"))
    torch.cuda.synchronize()
    arrivals = np.array([r["arrival"] for r in reqs]) - reqs[0]["arrival"]

    def make(dst):
        return lambda r: dict(geom=reqs[r]["geometry"], y=ys[r], out=dst[r], lam=cfg["lam"],
                              iters=tuple(cfg["iters"]))

    res = {"requests": n_requests, "budget_bytes": cfg["budget_bytes"], "iters": cfg["iters"][0]}
    for name, arr in (("plain", arrivals), ("plain_saturated", np.zeros_like(arrivals))):
        log("serving: %s (one at a time)" % name)
        lat, span = plain_replay(arr, reqs, make(ref))
        res[name] = summarize(lat, span)
    for name, arr in (("served", arrivals), ("served_saturated", np.zeros_like(arrivals))):
        log("serving: %s (8 slots)" % name)
        srv = Server(budget_bytes=cfg["budget_bytes"], max_slots=8)
        # first-request costs (plan tables, Schur step) are part of serving
        lat, span, _ = replay(srv, arr, make(outs))
        st = srv.stats()
        launches, items = srv.batch_stats()
        srv.close()
        same = all(torch.equal(a, b) for a, b in zip(outs, ref))
        res[name] = dict(summarize(lat, span), peak_running=st["peak_running"],
                         peak_device_gb=st["peak_in_use"] / 1e9, batched_launches=launches,
                         items_per_launch=items / max(launches, 1), bitwise_equal_to_plain=same)
    res["throughput_gain_saturated"] = res["served_saturated"]["req_per_s"] / res["plain_saturated"]["req_per_s"]
    return res


def operator_table():
    """P (cbct_forward, with its copy of the volume into z-contiguous columns) and P^T
    (cbct_adjoint) at each configuration and level: the 32^3 / 16-view cube, both levels of the
    512x512x64 / 40-view benchmark and the 8 x 128^3 / 60-view batch (one call per volume), on
    seeded uniform volumes and projections.  HIP events on the stream they run on, 3 warm-ups,
    then the median and 90th percentile of 20 runs; voxel.views/s from the median."""
    import numpy as np
    import torch

    import cbct_synth as S
    from paper_1001_0599_amd.ops import Plan

    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    cases = (("cube32", S.CONFIGS["cube32"], (0,), 1), ("wide512x512x64", S.CONFIGS["wide512x512x64"], (0, 1), 1),
             ("batch8x128", S.CONFIGS["batch8x128"], (0,), S.CONFIGS["batch8x128"]["batch"]))
    res = {}
    for name, c, lvls, batch in cases:
        g = c["geometry"]
        plan = Plan(g, levels=c.get("levels", 1))
        for lvl in lvls:
            vs, ps = plan.vol_shape(lvl), plan.proj_shape(lvl)
            f = torch.rand((batch,) + vs, device="cuda", generator=gen) * 0.02
            y = torch.rand((batch,) + ps, device="cuda", generator=gen)
            p, v = torch.empty_like(y), torch.empty_like(f)
            fws = torch.empty(plan.forward_workspace_bytes(lvl), dtype=torch.uint8, device="cuda")
            aws = torch.empty(plan.adjoint_workspace_bytes(lvl), dtype=torch.uint8, device="cuda")

            def fwd():
                for b in range(batch):
                    plan.forward(f[b], level=lvl, out=p[b], workspace=fws)

            def adj():
                for b in range(batch):
                    plan.adjoint(y[b], level=lvl, out=v[b], workspace=aws)

            row = {"volume": "x".join(str(n) for n in vs[::-1]) + ("" if batch == 1 else " x %d" % batch),
                   "views": ps[0], "detector": "%dx%d" % (ps[2], ps[1])}
            vv = batch * vs[0] * vs[1] * vs[2] * ps[0]
            for op, fn in (("P", fwd), ("P^T", adj)):
                for _ in range(3):
                    fn()
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
                for e0, e1 in ev:
                    e0.record()
                    fn()
                    e1.record()
                torch.cuda.synchronize()
                ms = np.array([a.elapsed_time(b) for a, b in ev])
                med, p90 = float(np.median(ms)), float(np.percentile(ms, 90))
                row[op] = {"median_ms": med, "p90_ms": p90, "voxel_views_per_s": vv / (med * 1e-3)}
            res["%s level %d" % (name, lvl)] = row
            del f, y, p, v, fws, aws
    return res


def small_solves():
    """Solves that are bound by launches and the ROF loop's decisions rather than by bandwidth:
    the 32^3 / 16-view cube (20 iterations), the low-dose 32^3 sweep (3 levels x 100 iterations,
    lambda 0.02 / 0.05 / 0.1, I0 = 2e3) and a 128^3 / 60-view volume (20 iterations, its ROF loop
    on gated launch chains); and the autograd loss of the 8 x 128^3 batch with its backward pass.
    Milliseconds per solve (or loss and backward), medians of repeats."""
    import numpy as np
    import torch

    import cbct_synth as S
    from paper_1001_0599_amd.ops import Plan

    def timed(plan, y, lam, iters, reps):
        out = torch.empty(plan.vol_shape(0), device="cuda")
        plan.reconstruct(y, lam=lam, iters=iters, out=out)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            plan.reconstruct(y, lam=lam, iters=iters, out=out)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)) * 1e3

    def noisy(g, seeds, i0):
        ph = S.make_phantom(g, seeds[0])
        return S.poisson_log_torch(S.analytic_projections_torch(g, ph, "cuda"), i0, seeds[1]).float().contiguous()

    res = {}
    c = S.CONFIGS["cube32"]
    res["cube32_16views_20it_ms"] = timed(Plan(c["geometry"], levels=1), noisy(c["geometry"], c["seeds"], c["I0"]),
                                         c["lam"], c["iters"], 20)
    c = S.CONFIGS["lowdose32"]
    plan = Plan(c["geometry"], levels=c["levels"])
    y = noisy(c["geometry"], c["seeds"], c["I0"])
    res["lowdose32_3x100it_ms"] = {str(lam): timed(plan, y, lam, c["iters"], 3) for lam in c["lam"]}
    g = S.CONFIGS["batch8x128"]["geometry"]
    res["vol128_60views_20it_ms"] = timed(Plan(g, levels=1), noisy(g, (41, 49), 1e5), 0.05, [20], 5)
    # the autograd loss of the 8 x 128^3 batch: sum (P f - y)^2 + lambda TV(f), forward and backward
    from paper_1001_0599_amd.autograd import project, tv_sum
    c = S.CONFIGS["batch8x128"]
    plan = Plan(g, levels=1)
    torch.manual_seed(0)
    f = (0.02 * torch.rand((c["batch"],) + tuple(g.vol_shape), device="cuda")).requires_grad_(True)
    y = torch.rand((c["batch"],) + tuple(g.proj_shape), device="cuda")

    def step():
        f.grad = None
        r = project(f, plan) - y
        ((r * r).sum() + c["lam"] * tv_sum(f, plan)).backward()

    step()
    torch.cuda.synchronize()
    ts = []
    for _ in range(10):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    res["autograd_8x128_loss_backward_ms"] = float(np.median(ts)) * 1e3
    return res


def kernels_only():
    """One launch each of a plain 256 MB copy and the hot kernels at the 512x512x64 / 40-view size:
    P (k_forward_runs), P^T (k_adj_profiles, k_adj_gather_staged, k_adj_combine), the Eq. 6 backprojector, the
    Siddon pair, and the TV passes (k_tv_grad, k_tv_trial<1>); the driver for hardware-counter
    runs, whose records `--counter-summary` turns into the traffic and L2 hit-rate table."""
    import torch

    import cbct_synth as S
    from paper_1001_0599_amd.ops import Plan

    torch.cuda.set_device(0)
    g = S.config_geometry("wide512x512x64")
    plan = Plan(g, levels=1)
    ph = S.make_phantom(g, 21)
    y = S.poisson_log_torch(S.analytic_projections_torch(g, ph, "cuda"), 1e5, 22).float().contiguous()
    f_cols = torch.rand((g.ny, g.nx, g.nz), device="cuda") * 0.02
    proj = torch.empty_like(y)
    vol = torch.empty(g.vol_shape, device="cuda")
    a = torch.empty(64 * 2 ** 20, device="cuda")
    b = torch.empty_like(a)
    zws = torch.empty(plan.adjoint_workspace_bytes(0), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    b.copy_(a)
    plan.forward_columns(f_cols, out=proj)
    plan.adjoint(y, out=vol, workspace=zws)
    plan.backproject_eq6(y, out=vol)
    del zws
    sws = torch.empty(max(plan.forward_workspace_bytes(0), plan.adjoint_siddon_workspace_bytes(0)),
                      dtype=torch.uint8, device="cuda")
    fv = f_cols.permute(2, 0, 1).contiguous()
    plan.forward_siddon(fv, out=proj, workspace=sws)
    plan.adjoint_siddon(y, out=vol, workspace=sws)
    del sws
    # the TV passes: one gradient pass, and one ROF iteration of the host-driven loop (a replayed
    # decision selects it): gradient, the first trial window, decision, update
    plan.tv_energy_grad(fv)
    plan.tv_prox(fv, 0.05, 1e-3, replay=[(0, 1)])
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 2 * 4 * a.numel()}))


COUNTER_KERNELS = [  # (label, kernel-name prefix) in the order of the table
    ("device copy (256 MiB, calibration)", "__amd_rocclr_copyBuffer"),
    ("P: k_forward_runs", "k_forward_runs"),
    ("P^T pass 1: k_adj_profiles", "k_adj_profiles"),
    ("P^T pass 2: k_adj_gather_staged", "k_adj_gather_staged"),
    ("P^T view-group sum: k_adj_combine", "k_adj_combine"),
    ("Eq. 6: k_backproject_eq6", "k_backproject_eq6"),
    ("P_s: k_siddon_forward_runs", "k_siddon_forward_runs"),
    ("P_s^T pass 1: k_sid_profiles", "k_sid_profiles"),
    ("P_s^T pass 2: k_sid_gather_pieces", "k_sid_gather_pieces"),
    ("Step 2: k_tv_grad", "k_tv_grad"),
    ("Step 2: k_tv_trial", "k_tv_trial"),
]


def read_counters(d, names):
    """Per kernel and counter, the values of its dispatches (each summed over the counter's
    instances), from a rocprofv3 output directory (its SQLite database)."""
    import glob
    import re
    import sqlite3
    from collections import defaultdict

    dbs = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
    if not dbs:
        raise SystemExit("no rocprofv3 database under %s" % d)
    con = sqlite3.connect(dbs[0])
    per = defaultdict(lambda: defaultdict(float))  # kernel -> dispatch -> sum over the names
    for disp, kn, cn, v in con.execute(
            "select dispatch_id, kernel_name, counter_name, value from counters_collection"):
        if cn not in names:
            continue
        k = re.sub(r"\(.*", "", kn.replace("void ", "").replace("(anonymous namespace)::", ""))
        per[(k, cn)][disp] += v
    return {key: list(by_disp.values()) for key, by_disp in per.items()}


def counter_summary(fetch_dir, write_dir, hit_dir):
    """Print the traffic and L2 hit-rate record (the file TRAFFIC_RECORD holds) from three counter
    runs of --kernels-only."""
    F = read_counters(fetch_dir, {"FETCH_SIZE"})
    W = read_counters(write_dir, {"WRITE_SIZE"})
    H = read_counters(hit_dir, {"TCC_HIT_sum", "TCC_MISS_sum"})

    def pick(tab, prefix, cn):
        # the mean over the kernel's dispatches; for the copy, its largest dispatch (the 256 MiB
        # calibration copy, not the small copies around it)
        vals = [v for (k, c), v in tab.items()
                if c == cn and (k == prefix or k.startswith(prefix + "<") or k.startswith(prefix + "("))]
        if len(vals) != 1:
            return None
        return max(vals[0]) if prefix == COUNTER_KERNELS[0][1] else sum(vals[0]) / len(vals[0])

    copy_half = 64 * 2 ** 20 * 4  # bytes the copy reads (and writes)
    cf = copy_half / (pick(F, COUNTER_KERNELS[0][1], "FETCH_SIZE") * 1024)
    cw = copy_half / (pick(W, COUNTER_KERNELS[0][1], "WRITE_SIZE") * 1024)
    rows, got = [], {}
    for label, pre in COUNTER_KERNELS:
        fs, ws = pick(F, pre, "FETCH_SIZE"), pick(W, pre, "WRITE_SIZE")
        hi, mi = pick(H, pre, "TCC_HIT_sum"), pick(H, pre, "TCC_MISS_sum")
        if fs is None or ws is None:
            continue
        gb = (fs * 1024 * cf + ws * 1024 * cw) / 1e9
        hit = hi / (hi + mi) if hi is not None and mi is not None and hi + mi > 0 else float("nan")
        got[pre] = (gb, hi or 0.0, mi or 0.0)
        rows.append("  %-36s %14.1f %14.1f %10.3f %9.1f%%" % (label, fs, ws, gb, 100 * hit))
    pt_kernels = [k for k in ("k_adj_profiles", "k_adj_gather_staged", "k_adj_combine") if k in got]
    pt_gb = sum(got[k][0] for k in pt_kernels)
    pt_hit = sum(got[k][1] for k in pt_kernels)
    pt_miss = sum(got[k][2] for k in pt_kernels)
    lines = [
        "HBM traffic and L2 hit rate per launch from hardware counters, 512x512x64 voxels, 40 views,",
        "512x384 detector (MI355X, gfx950).  Three rocprofv3 runs of the same program, from the repository root:",
        "  cd /tmp && export TMPDIR=/tmp",
        "  rocprofv3 --pmc FETCH_SIZE --kernel-trace -d <fetch> -o run -- python3 <repo>/bench.py --kernels-only",
        "  rocprofv3 --pmc WRITE_SIZE --kernel-trace -d <write> -o run -- python3 <repo>/bench.py --kernels-only",
        "  rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum --kernel-trace -d <hit> -o run -- python3 <repo>/bench.py --kernels-only",
        "  python3 bench.py --counter-summary <fetch> <write> <hit> > profiles/adjoint_traffic_512x512x64_40views.txt",
        "FETCH_SIZE and WRITE_SIZE are scaled by (bytes a plain 256 MiB device copy moves) / (what the counter",
        "reads for that copy); L2 hit rate = TCC_HIT / (TCC_HIT + TCC_MISS).  Values are means per dispatch.",
        "",
        "  %-36s %14s %14s %10s %10s" % ("kernel", "FETCH_SIZE KiB", "WRITE_SIZE KiB", "HBM GB", "L2 hit"),
    ] + rows + [
        "",
        "  copy calibration: FETCH x %.3f, WRITE x %.3f" % (cf, cw),
        "",
        "Machine-readable (bench.py reports hbm_bytes_per_launch as roofline.traffic and the L2 hit rate",
        "while the digest of %s still matches):" % ", ".join(TRAFFIC_SOURCES),
        "kernel: " + " + ".join(pt_kernels),
        "hbm_bytes_per_launch: %.0f" % (pt_gb * 1e9),
        "l2_hit_rate: %.4f" % (pt_hit / (pt_hit + pt_miss)),
        "forward_hbm_bytes_per_launch: %.0f" % (got["k_forward_runs"][0] * 1e9),
        "sources_sha256: %s" % sources_digest(TRAFFIC_SOURCES),
    ]
    print("\n".join(lines))


SQ_KERNELS = ["k_forward_runs", "k_adj_profiles", "k_adj_gather_staged", "k_adj_combine",
              "k_backproject_eq6", "k_siddon_forward_runs", "k_sid_profiles", "k_sid_gather_pieces", "k_tv_grad",
              "k_tv_trial", "k_sum_rows"]


def sq_summary(d):
    """Instruction-mix record of the hot kernels from one rocprofv3 run of --kernels-only with the
    SQ counters (wave-level instruction counts, LDS bank-conflict cycles, busy and wave cycles) and
    the kernel durations of the same run."""
    import glob
    import re
    import sqlite3
    from collections import defaultdict

    names = ["SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
             "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES", "SQ_WAVES"]
    tab = {n: read_counters(d, {n}) for n in names}
    dbs = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
    con = sqlite3.connect(dbs[0])
    dur = defaultdict(list)
    for name, du in con.execute("select name, duration from kernels"):
        k = re.sub(r"\(.*", "", name.replace("void ", "").replace("(anonymous namespace)::", ""))
        dur[k].append(du)

    def pick(t, pre):
        vals = [v for (k, c), v in t.items() if k == pre or k.startswith(pre + "<")]
        return sum(vals[0]) / len(vals[0]) if len(vals) == 1 else None

    def dpick(pre):
        v = [x for k, xs in dur.items() if k == pre or k.startswith(pre + "<") for x in xs]
        return sum(v) / len(v) if v else None

    peak_issue = 256 * 2.4e9  # VALU wave-instructions per second: 256 CUs, one per clock each
    lines = [
        "Instruction mix of the hot kernels, 512x512x64 voxels, 40 views, 512x384 detector (MI355X, gfx950).",
        "One rocprofv3 run of the same program, from the repository root:",
        "  cd /tmp && export TMPDIR=/tmp",
        "  rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
        "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_WAVES --kernel-trace -d <dir> -o run -- python3 <repo>/bench.py "
        "--kernels-only",
        "  python3 bench.py --sq-summary <dir>",
        "Counts are per dispatch (means over the kernel's dispatches), wave-level instructions.  'VALU at peak' is",
        "SQ_INSTS_VALU / (256 CUs x 2.4 GHz x 1 wave-instruction per CU per clock): the time the kernel would take",
        "if VALU issue were its only limit; 'VALU share' is that over the kernel's duration in this run.",
        "",
        "  %-26s %12s %10s %12s %11s %9s %10s %9s" % ("kernel", "VALU instr", "LDS instr", "bank confl",
                                                    "confl/LDS", "dur us", "VALU@pk us", "VALU shr"),
    ]
    for k in SQ_KERNELS:
        va, ld, bc = pick(tab["SQ_INSTS_VALU"], k), pick(tab["SQ_INSTS_LDS"], k), pick(tab["SQ_LDS_BANK_CONFLICT"], k)
        du = dpick(k)
        if va is None or du is None:
            continue
        t_pk = va / peak_issue * 1e6
        lines.append("  %-26s %12.4g %10.4g %12.4g %11.2f %9.1f %10.1f %8.0f%%" % (
            k, va, ld or 0, bc or 0, (bc or 0) / ld if ld else 0.0, du / 1e3, t_pk, 100 * t_pk / (du / 1e3)))
    print("\n".join(lines))


def trace_summary(d, top=40):
    """Per kernel and launch grid: calls, total / mean / min / max duration, share, VGPRs and LDS,
    from the kernel trace in a rocprofv3 output directory (its SQLite database)."""
    import glob
    import re
    import sqlite3
    from collections import defaultdict

    dbs = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
    if not dbs:
        raise SystemExit("no rocprofv3 database under %s" % d)
    con = sqlite3.connect(dbs[0])
    acc, meta = defaultdict(list), {}
    for name, dur, vg, lds, gx, gy, gz in con.execute(
            "select name, duration, vgpr_count, lds_size, grid_x, grid_y, grid_z from kernels"):
        n = re.sub(r"^void ", "", name).replace("(anonymous namespace)::", "")
        n = re.sub(r"\((float|double|int|long|unsigned|ColParams|RofControl|AdjArgs|SidArgs|SidCol|const|ZIndex|"
                   r"ViewParams).*$", "", n)
        n = "%s [%dx%dx%d]" % (n, gx, gy, gz)
        acc[n].append(dur)
        meta[n] = (vg, lds)
    tot = sum(sum(v) for v in acc.values())
    w = 62
    print("%-*s %6s %9s %9s %8s %8s %6s %5s %6s" % (w, "kernel", "calls", "total ms", "mean us", "min us", "max us", "%",
                                                 "vgpr", "lds"))
    for n, v in sorted(acc.items(), key=lambda kv: -sum(kv[1]))[:top]:
        vg, lds = meta[n]
        print("%-*s %6d %9.3f %9.2f %8.2f %8.2f %6.2f %5d %6d" % (w, n[:w], len(v), sum(v) / 1e6, sum(v) / len(v) / 1e3,
                                                              min(v) / 1e3, max(v) / 1e3, 100 * sum(v) / tot, vg, lds))
    print("all kernels: %.3f ms" % (tot / 1e6))


def occupancy_run(which):
    """A workload for a GPU-busy record under a rocprofv3 kernel trace: warm-up passes (plans,
    cached Schur steps and workspaces in place), a 0.5 s pause that marks the window, then timed
    passes back to back.  'recon': three 512x512x64 / 40-view reconstructions; 'cube32': five
    32^3 / 16-view solves; 'plain32': the plain one-at-a-time loop over the first 32 requests of
    the serving workload (one plan per geometry, each warmed once)."""
    import torch

    import cbct_synth as S
    from paper_1001_0599_amd.ops import Plan

    def noisy(g, seeds, i0):
        ph = S.make_phantom(g, seeds[0])
        return S.poisson_log_torch(S.analytic_projections_torch(g, ph, "cuda"), i0, seeds[1]).float().contiguous()

    jobs = []  # (plan, y, lam, iters, out)
    if which in ("recon", "cube32"):
        c = S.CONFIGS["wide512x512x64" if which == "recon" else "cube32"]
        g = c["geometry"]
        plan = Plan(g, levels=c["levels"])
        y = noisy(g, c["seeds"], c["I0"])
        out = torch.empty(plan.vol_shape(0), device="cuda")
        jobs = [(plan, y, c["lam"], tuple(c["iters"]), out)] * (3 if which == "recon" else 5)
        warm = jobs[:1]
    elif which == "plain32":
        cfg = S.CONFIGS["serving_mix"]
        plans, warm = {}, []
        for r in S.serving_requests(32):
            g = r["geometry"]
            key = (g.nx, g.ny, g.nz, g.n_views, g.nu, g.nv)
            y = noisy(g, (r["phantom_seed"], r["noise_seed"]), cfg["I0"])
            fresh = key not in plans
            if fresh:
                plans[key] = Plan(g)
            job = (plans[key], y, cfg["lam"], tuple(cfg["iters"]), torch.empty(g.vol_shape, device="cuda"))
            if fresh:
                warm.append(job)
            jobs.append(job)
    else:
        raise SystemExit("unknown occupancy workload %r (recon, cube32, plain32)" % which)
    for plan, y, lam, iters, out in warm:
        plan.reconstruct(y, lam=lam, iters=iters, out=out)
    torch.cuda.synchronize()
    time.sleep(0.5)
    t0 = time.perf_counter()
    for plan, y, lam, iters, out in jobs:
        plan.reconstruct(y, lam=lam, iters=iters, out=out)
    torch.cuda.synchronize()
    print("%s: %d passes in %.2f ms (wall)" % (which, len(jobs), (time.perf_counter() - t0) * 1e3), flush=True)


def busy_summary(d, passes, top=16):
    """GPU-busy record of an occupancy run's kernel trace: the window is everything after the
    trace's longest gap between kernels (the run's pause); busy time is the union of the kernels'
    intervals in it, against the window from the first kernel's start to the last one's end."""
    import glob
    import re
    import sqlite3
    from collections import defaultdict

    dbs = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
    if not dbs:
        raise SystemExit("no rocprofv3 database under %s" % d)
    con = sqlite3.connect(dbs[0])
    cols = [r[1] for r in con.execute("pragma table_info(kernels)")]
    wgc = [next((c for c in cols if re.fullmatch(r"(workgroup|wg)(_size)?_%s" % ax, c)), None) for ax in "xyz"]
    sel = "name, start, end, grid_x, grid_y, grid_z" + ("".join(", " + c for c in wgc) if all(wgc) else "")
    rows = list(con.execute("select %s from kernels order by start" % sel))
    if len(rows) < 2:
        raise SystemExit("too few kernels in the trace")
    gi = max(range(len(rows) - 1), key=lambda i: rows[i + 1][1] - rows[i][2])
    win = rows[gi + 1:]
    t0, t1 = win[0][1], max(r[2] for r in win)
    busy, cs, ce = 0, None, None
    for _, st, en, *_ in win:
        if ce is None or st > ce:
            if ce is not None:
                busy += ce - cs
            cs, ce = st, en
        else:
            ce = max(ce, en)
    busy += ce - cs
    ksum = sum(en - st for _, st, en, *_ in win)
    print("window %.3f ms (first kernel start to last kernel end), GPU busy %.3f ms = %.1f %%" % (
        (t1 - t0) / 1e6, busy / 1e6, 100.0 * busy / (t1 - t0)))
    print("kernels %d (%.1f per pass over %d passes), summed durations %.3f ms, mean %.2f us" % (
        len(win), len(win) / passes, passes, ksum / 1e6, ksum / len(win) / 1e3))
    if all(wgc):
        # launches by work-group count: 256 CUs hold at least 2 work-groups of 256 lanes each
        bins = [(0, 256), (256, 1024), (1024, 4096), (4096, 1 << 62)]
        tb = [0] * len(bins)
        for _, st, en, gx, gy, gz, wx, wy, wz in win:
            nwg = -(-gx // max(wx, 1)) * -(-gy // max(wy, 1)) * -(-gz // max(wz, 1))
            tb[next(i for i, (lo, hi) in enumerate(bins) if lo <= nwg < hi)] += en - st
        print("kernel time by launch size: " + ", ".join(
            "%s work-groups %.1f %%" % ("%d-%d" % (lo, hi - 1) if hi < 1 << 62 else ">= %d" % lo, 100.0 * t / ksum)
            for (lo, hi), t in zip(bins, tb)))
    else:
        print("(no work-group size columns in the trace's kernel table: %s)" % ", ".join(cols))
    agg = defaultdict(lambda: [0, 0])
    for n, st, en, *_ in win:
        k = re.sub(r"^void ", "", n).replace("(anonymous namespace)::", "")
        k = re.sub(r"\(.*", "", k)
        agg[k][0] += en - st
        agg[k][1] += 1
    print("%-46s %7s %10s %9s" % ("kernel", "calls", "total ms", "mean us"))
    for k, (du, c) in sorted(agg.items(), key=lambda kv: -kv[1][0])[:top]:
        print("%-46s %7d %10.3f %9.2f" % (k[:46], c, du / 1e6, du / c / 1e3))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving", type=int, default=256, metavar="N",
                    help="requests of the serving workload to replay (256 in the full workload; 0: skip)")
    ap.add_argument("--kernels-only", action="store_true", help="one launch of each hot kernel (for counters)")
    ap.add_argument("--counter-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "HIT_DIR"),
                    help="print the traffic / L2 hit-rate record from three counter runs of --kernels-only")
    ap.add_argument("--trace-summary", metavar="DIR", help="per-kernel table of a rocprofv3 kernel-trace run")
    ap.add_argument("--sq-summary", metavar="DIR", help="instruction-mix record from a rocprofv3 SQ-counter run")
    ap.add_argument("--occupancy", choices=("recon", "cube32", "plain32"),
                    help="run one workload for a GPU-busy kernel trace (see --busy-summary)")
    ap.add_argument("--busy-summary", nargs=2, metavar=("DIR", "PASSES"),
                    help="GPU-busy record of a rocprofv3 kernel trace of an --occupancy run")
    args = ap.parse_args()
    if args.occupancy:
        occupancy_run(args.occupancy)
        return
    if args.busy_summary:
        busy_summary(args.busy_summary[0], int(args.busy_summary[1]))
        return
    if args.counter_summary:
        counter_summary(*args.counter_summary)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.sq_summary:
        sq_summary(args.sq_summary)
        return
    if args.kernels_only:
        kernels_only()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (it times the one-GPU "
              "share of the workload); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import cbct_synth as S
    from paper_1001_0599_amd.ops import Plan

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    cfg = S.CONFIGS["wide512x512x64"]
    g = cfg["geometry"]
    iters = cfg["iters"]
    lam = cfg["lam"]
    log("generating the seeded ellipsoid phantom and its noisy projections")
    ph = S.make_phantom(g, cfg["seeds"][0])
    Y = torch.tensor(S.poisson_log(S.analytic_projections(g, ph), cfg["I0"], cfg["seeds"][1]), dtype=torch.float32,
                     device=dev)
    plan = Plan(g, levels=cfg["levels"])
    params, keep = plan.solve_params(lam, iters)
    ws = torch.empty(plan.reconstruct_workspace_bytes(params), dtype=torch.uint8, device=dev)
    out = torch.empty(plan.vol_shape(0), dtype=torch.float32, device=dev)

    log("warm-up (includes the Schur-bound step estimate, cached in the plan)")
    t0 = time.perf_counter()
    plan.reconstruct(Y, lam=lam, iters=iters, out=out, workspace=ws)
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t0
    for _ in range(args.warmup - 1):
        plan.reconstruct(Y, lam=lam, iters=iters, out=out, workspace=ws)
    torch.cuda.synchronize()

    log("timed reconstructions")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.reconstruct(Y, lam=lam, iters=iters, out=out, workspace=ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    recon_s = wall / args.steps
    # P / P^T applications per reconstruction: one of each per outer iteration per level
    vv_job = 0
    for lvl, it in enumerate(iters):
        nz, ny, nx = plan.vol_shape(lvl)
        vv_job += 2 * it * nx * ny * nz * g.n_views

    # per-kernel rates at the finest level: the projector kernel alone on a column-major
    # volume (as inside the solver) and the adjoint gather, timed with HIP events on the
    # stream they run on
    log("per-operator timing")
    f_cols = out.permute(1, 2, 0).contiguous()
    proj = torch.empty(plan.proj_shape(0), dtype=torch.float32, device=dev)
    vol = torch.empty(plan.vol_shape(0), dtype=torch.float32, device=dev)
    zws = torch.empty(plan.adjoint_workspace_bytes(0), dtype=torch.uint8, device=dev)
    for _ in range(3):
        plan.forward_columns(f_cols, out=proj)
        plan.adjoint(Y, out=vol, workspace=zws)
    n_ev = 20
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(n_ev)]
    for e0, e1, e2 in ev:
        e0.record()
        plan.forward_columns(f_cols, out=proj)
        e1.record()
        plan.adjoint(Y, out=vol, workspace=zws)
        e2.record()
    torch.cuda.synchronize()
    tp = float(np.mean([a.elapsed_time(b) for a, b, _ in ev])) * 1e-3
    ta = float(np.mean([b.elapsed_time(c) for _, b, c in ev])) * 1e-3
    # the paper's Eq. 6 backprojector alone, and the reconstruction with it in Step 1
    for _ in range(3):
        plan.backproject_eq6(Y, out=vol)
    ev6 = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(n_ev)]
    for e0, e1 in ev6:
        e0.record()
        plan.backproject_eq6(Y, out=vol)
        e1.record()
    torch.cuda.synchronize()
    tb6 = float(np.mean([a.elapsed_time(b) for a, b in ev6])) * 1e-3
    # the Siddon pair (exact ray-in-voxel lengths) at the same size
    sws = torch.empty(max(plan.forward_workspace_bytes(0), plan.adjoint_siddon_workspace_bytes(0)), dtype=torch.uint8,
                      device=dev)
    for _ in range(2):
        plan.forward_siddon(out, out=proj, workspace=sws)
        plan.adjoint_siddon(Y, out=vol, workspace=sws)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(10)]
    for e0, e1, e2 in evs:
        e0.record()
        plan.forward_siddon(out, out=proj, workspace=sws)
        e1.record()
        plan.adjoint_siddon(Y, out=vol, workspace=sws)
        e2.record()
    torch.cuda.synchronize()
    tps = float(np.mean([a.elapsed_time(b) for a, b, _ in evs])) * 1e-3
    tas = float(np.mean([b.elapsed_time(c) for _, b, c in evs])) * 1e-3
    del sws
    def recon_variant(**kw):
        """Seconds per reconstruction with other solver options (a warm-up call caches the
        pair's Schur step first)."""
        params, keep = plan.solve_params(lam, iters, **kw)
        wsv = torch.empty(plan.reconstruct_workspace_bytes(params), dtype=torch.uint8, device=dev)
        plan.reconstruct(Y, lam=lam, iters=iters, out=out, workspace=wsv, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = max(1, min(args.steps, 3))
        for _ in range(n):
            plan.reconstruct(Y, lam=lam, iters=iters, out=out, workspace=wsv, **kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    log("reconstruction variants: Eq. 6 Step 1, Siddon pair, Siddon + Eq. 6")
    recon6_s = recon_variant(step1_eq6=True)
    recon_sid_s = recon_variant(projector=1)
    recon_sid6_s = recon_variant(projector=1, step1_eq6=True)
    vv = g.n_vox * g.n_views
    # algorithmic bytes per launch: the volume read (P) or written (P^T) once per view, plus the
    # detector samples in and out (4 B each)
    alg_bytes = 4.0 * vv + 8.0 * g.n_views * g.nu * g.nv
    # the dominant operator: P^T (two launches, z profiles then the gather) or P (one launch)
    if ta >= tp:
        dom, t_dom = "P^T: k_adj_profiles + k_adj_gather_staged + k_adj_combine", ta
        traffic, l2_hit = measured_traffic()
    else:
        dom, t_dom, traffic, l2_hit = "P: k_forward_runs", tp, None, None
    achieved = alg_bytes / t_dom / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "l2_hit_rate": l2_hit, "kernel": dom,
                "kernel_ms": t_dom * 1e3, "bytes_per_launch": alg_bytes}

    res = {
        "metric": "P/P^T voxel·views/s, recon s @512²×64/40 views, served p50/p99 vs plain",
        "value": vv_job / recon_s,
        "unit": "voxel·views/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": recon_s * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "FBS-TV reconstruction, 512x512x64 voxels (0.9x0.9x2.5 mm), 40 views over 360 deg, "
                               "512x384 detector (0.78 mm), SAD 1000 / SDD 1536 mm, seeded ellipsoid phantom, "
                               "I0 = 1e5 Poisson",
                   "levels": cfg["levels"], "iters": iters, "lambda": lam},
        "recon_s": recon_s,
        "first_recon_s_incl_schur_probe": first_s,
        "p_voxel_views_per_s": vv / tp, "pt_voxel_views_per_s": vv / ta,
        "p_ms": tp * 1e3, "pt_ms": ta * 1e3,
        "eq6_backprojector_ms": tb6 * 1e3, "recon_s_step1_eq6": recon6_s,
        "siddon_p_ms": tps * 1e3, "siddon_pt_ms": tas * 1e3,
        "recon_s_siddon_pair": recon_sid_s, "recon_s_siddon_p_eq6_step1": recon_sid6_s,
        "roofline": roofline,
    }
    log("launch-bound solves: 32^3, low-dose 32^3 sweep, 128^3")
    res["solves"] = small_solves()
    log("per-operator table: cbct_forward / cbct_adjoint per configuration and level")
    res["operators"] = operator_table()
    if args.serving:
        res["serving"] = serving_run(args.serving)
    if not args.no_cpu_baseline:
        log("CPU oracle baseline (bounded sample)")
        cb = cpu_baseline(g, iters, lam)
        cb["host"] = host_cpu()
        # the same rate on the GPU (P and P^T at the fine level) and the same job, over the oracle's
        gpu_pair = 2.0 * vv / (tp + ta)
        cb["gpu_over_oracle"] = gpu_pair / cb["value"]
        cb["gpu_over_oracle_1thread"] = gpu_pair / cb["value_1thread"]
        cb["recon_gpu_over_oracle_extrapolated"] = cb["recon_s_extrapolated"] / recon_s
        res["cpu_baseline"] = cb
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
