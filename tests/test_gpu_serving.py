"""The serving runtime on the GPU: a mix of requests admitted concurrently under an HBM budget;
every result is bitwise equal to the same request solved alone (cbct_reconstruct); the budget
is respected; latencies are reported."""
import dataclasses

import numpy as np
import pytest
import torch

import cbct_synth as S
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _requests():
    base = S.config_geometry("cube32")
    geos = [dataclasses.replace(base, n_views=nv, nx=n, ny=n, nz=nz, nu=2 * n, nv=2 * nz)
            for nv, n, nz in ((16, 32, 32), (24, 48, 32), (12, 32, 16), (20, 64, 32), (16, 32, 32), (30, 48, 16))]
    reqs = []
    for r, g in enumerate(geos):
        ph = S.make_phantom(g, 5000 + r)
        p = S.analytic_projections_torch(g, ph, "cuda")
        y = S.poisson_log_torch(p, 1e5, 6000 + r).float().contiguous()
        reqs.append((g, y))
    return reqs


def test_mixed_requests_equal_solo_results():
    from paper_1001_0599_amd.ops import Plan
    from paper_1001_0599_amd.serving import Server
    announce("serving: 6 mixed requests, 4 slots")
    reqs = _requests()
    solo = []
    for g, y in reqs:
        solo.append(Plan(g).reconstruct(y, lam=0.05, iters=[10]))
    torch.cuda.synchronize()
    srv = Server(budget_bytes=4e9, max_slots=4)
    outs = [torch.empty(g.vol_shape, device="cuda") for g, _ in reqs]
    tickets = []
    for q, ((g, y), o) in enumerate(zip(reqs, outs)):
        # every other request hands its projections over from host memory
        yin = y.cpu().numpy() if q % 2 else y
        tickets.append(srv.submit(g, yin, o, lam=0.05, iters=(10,)))
    srv.wait_all()
    st = srv.stats()
    # peak_in_use: the device bytes the server obtained (pool blocks and plan tables)
    assert st["completed"] == len(reqs) and 0 < st["peak_in_use"] <= 4e9
    for t, o, s in zip(tickets, outs, solo):
        done, status, lat = srv.poll(t)
        assert done and status == 0 and lat > 0
        assert torch.equal(o, s)
    # the engine's launches carried several requests' work-groups
    launches, items = srv.batch_stats()
    assert launches > 0 and items > launches, (launches, items)
    srv.close()


def test_mixed_operator_choices_equal_solo_results():
    """Requests with the Siddon pair, Siddon P + Eq. 6, and the trilinear pair in one mix: each
    result equals its solo solve bitwise, and the admission estimate covers the Siddon tables."""
    from paper_1001_0599_amd.ops import Plan
    from paper_1001_0599_amd.serving import Server
    announce("serving: 6 requests, three operator choices, 3 slots")
    reqs = _requests()
    kws = [dict(projector=1), dict(projector=1, step1_eq6=1), dict()] * 2
    solo = [Plan(g).reconstruct(y, lam=0.05, iters=[6], **kw) for (g, y), kw in zip(reqs, kws)]
    torch.cuda.synchronize()
    srv = Server(budget_bytes=4e9, max_slots=3)
    outs = [torch.empty(g.vol_shape, device="cuda") for g, _ in reqs]
    tickets = [srv.submit(g, y, o, lam=0.05, iters=(6,), **kw) for (g, y), o, kw in zip(reqs, outs, kws)]
    srv.wait_all()
    for t, o, s in zip(tickets, outs, solo):
        done, status, _ = srv.poll(t)
        assert done and status == 0, srv.poll(t)
        assert torch.equal(o, s)
    srv.close()


def test_multilevel_requests_equal_solo_results():
    """Two-level requests through the batch engines: the coarse level of a 32^3 request (16^3)
    runs Step 2 in one work-group and its fine level as gated steps, larger ones gated on both
    levels; every result equals its solo solve bitwise."""
    from paper_1001_0599_amd.ops import Plan
    from paper_1001_0599_amd.serving import Server
    announce("serving: 4 two-level requests, 4 slots")
    reqs = _requests()[:4]
    iters = (3, 5)
    solo = [Plan(g, levels=2).reconstruct(y, lam=0.05, iters=list(iters)) for g, y in reqs]
    torch.cuda.synchronize()
    srv = Server(budget_bytes=4e9, max_slots=4)
    outs = [torch.empty(g.vol_shape, device="cuda") for g, _ in reqs]
    tickets = [srv.submit(g, y, o, lam=0.05, iters=iters) for (g, y), o in zip(reqs, outs)]
    srv.wait_all()
    for t, o, s in zip(tickets, outs, solo):
        done, status, _ = srv.poll(t)
        assert done and status == 0, srv.poll(t)
        assert torch.equal(o, s)
    srv.close()


def test_budget_serialises_when_tight():
    from paper_1001_0599_amd.serving import Server
    reqs = _requests()[:3]
    # one slot: the peak is the largest single request
    srv = Server(budget_bytes=1e12, max_slots=1)
    for g, y in reqs:
        srv.submit(g, y, torch.empty(g.vol_shape, device="cuda"), iters=(2,))
    srv.wait_all()
    one = srv.stats()["peak_in_use"]
    srv.close()
    srv = Server(budget_bytes=int(1.05 * one), max_slots=4)
    outs = []
    for g, y in reqs:
        outs.append(torch.empty(g.vol_shape, device="cuda"))
        srv.submit(g, y, outs[-1], iters=(2,))
    srv.wait_all()
    st = srv.stats()
    assert st["peak_in_use"] <= 1.05 * one
    srv.close()


def test_device_bytes_stay_within_budget():
    """Real device bytes (pooled blocks, idle ones included, and cached plan tables) never exceed
    the budget, also when many distinct geometries pass through (idle blocks and unused plans are
    given back), and a hipMemGetInfo drop taken while the server runs stays within it."""
    from paper_1001_0599_amd.serving import Server
    announce("serving: device bytes under a tight budget, 6 geometries")
    reqs = _requests()
    srv = Server(budget_bytes=1e12, max_slots=1)
    srv.submit(reqs[3][0], reqs[3][1], torch.empty(reqs[3][0].vol_shape, device="cuda"), iters=(1,))
    srv.wait_all()
    biggest = srv.stats()["peak_in_use"]
    srv.close()
    budget = int(1.6 * biggest)
    srv = Server(budget_bytes=budget, max_slots=4)
    outs = [torch.empty(g.vol_shape, device="cuda") for g, _ in reqs]
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    for (g, y), o in zip(reqs, outs):
        srv.submit(g, y, o, iters=(2,))
    low = free1
    while srv.stats()["completed"] < len(reqs):
        low = min(low, torch.cuda.mem_get_info()[0])
    srv.wait_all()
    st = srv.stats()
    assert st["peak_in_use"] <= budget, (st, budget)
    # allocation granularity aside (the runtime carves small tables out of larger chunks), what
    # the device lost is what the server holds
    assert free1 - low <= budget + (128 << 20), (free1 - low, budget)
    srv.close()
