"""Benchmark of the FBS-TV cone-beam reconstruction hot path on one MI355X.

Prints ONE JSON line.  See the design doc for the byte/flop models behind `roofline`.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the one-GPU share of a sharded solve is what it times)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import cbct_synth as S
    from paper_1001_0599_amd.ops import Plan

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    g = S.config_geometry("cfg2")
    plan = Plan(g, levels=2)
    ph = S.make_phantom(g, 21)
    f = torch.tensor(S.voxelize(g, ph, 1), dtype=torch.float32, device=dev)
    y = torch.tensor(S.poisson_log(S.analytic_projections(g, ph), 1e5, 22), dtype=torch.float32, device=dev)
    ws = torch.empty(plan.forward_workspace_bytes(0), dtype=torch.uint8, device=dev)
    proj = torch.empty_like(y)
    vol = torch.empty_like(f)

    def step():
        plan.forward(f, out=proj, workspace=ws)
        plan.adjoint(y, out=vol)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record()
        plan.forward(f, out=proj, workspace=ws)
        e1.record()
        plan.adjoint(y, out=vol)
        e2.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tp = float(np.median([a.elapsed_time(b) for a, b, _ in ev])) * 1e-3
    ta = float(np.median([b.elapsed_time(c) for _, b, c in ev])) * 1e-3
    vv = g.n_vox * g.n_views
    out = {
        "metric": "P/P^T voxel·views/s, recon s @512²×64/40 views, served p50/p99 vs plain",
        "value": 2 * vv / (tp + ta),
        "unit": "voxel·views/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "P+P^T pair, 512x512x64 voxels (0.9x0.9x2.5 mm), 40 views, 512x384 detector"},
        "p_s": tp, "pt_s": ta,
        "p_voxel_views_per_s": vv / tp, "pt_voxel_views_per_s": vv / ta,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
