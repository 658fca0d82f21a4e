"""The serving runtime's admission and slot logic (the C++ scheduler in simulated mode, host only):
FIFO order, the HBM budget is never exceeded, requests start while others run, oversize and
invalid requests are rejected at submit."""
import dataclasses
import time

import numpy as np
import pytest

import cbct_synth as S
from paper_1001_0599_amd import CbctError
from paper_1001_0599_amd.serving import Server

G = dataclasses.replace(S.config_geometry("cube32"), n_views=8)  # ~17 MB of workspace


def _bytes_one():
    srv = Server(budget_bytes=1e12, max_slots=1, simulated=True)
    srv.submit(G, iters=(1,), seconds=0.0)
    srv.wait_all()
    peak = srv.stats()["peak_in_use"]
    srv.close()
    return peak


def test_budget_limits_concurrency_and_order_is_fifo():
    one = _bytes_one()
    srv = Server(budget_bytes=2.5 * one, max_slots=8, simulated=True)  # room for two at a time
    tickets = [srv.submit(G, iters=(1,), seconds=0.05) for _ in range(8)]
    srv.wait_all()
    st = srv.stats()
    assert st["peak_in_use"] <= 2.5 * one
    assert st["peak_running"] == 2
    starts = [srv.times(t)[1] for t in tickets]
    assert starts == sorted(starts)
    srv.close()


def test_slots_limit_concurrency():
    srv = Server(budget_bytes=1e12, max_slots=3, simulated=True)
    for _ in range(9):
        srv.submit(G, iters=(1,), seconds=0.03)
    srv.wait_all()
    assert srv.stats()["peak_running"] == 3
    srv.close()


def test_late_arrivals_start_while_others_run():
    """Continuous admission: a request arriving during a long one starts before it ends."""
    srv = Server(budget_bytes=1e12, max_slots=4, simulated=True)
    t_long = srv.submit(G, iters=(1,), seconds=0.4)
    time.sleep(0.1)
    t_short = srv.submit(G, iters=(1,), seconds=0.05)
    srv.wait_all()
    long_t, short_t = srv.times(t_long), srv.times(t_short)
    assert short_t[1] < long_t[2] and short_t[2] < long_t[2]
    lat = srv.poll(t_short)[2]
    assert 0.04 < lat < 0.3
    srv.close()


def test_rejections():
    one = _bytes_one()
    srv = Server(budget_bytes=0.5 * one, max_slots=2, simulated=True)
    with pytest.raises(CbctError) as e:
        srv.submit(G, iters=(1,), seconds=0.0)
    assert e.value.status == 3  # CBCT_ERR_BUDGET
    with pytest.raises(CbctError) as e:
        srv.submit(dataclasses.replace(G, nx=0), iters=(1,))
    assert e.value.status == 1
    with pytest.raises(CbctError) as e:
        srv.submit(dataclasses.replace(G, nx=30), iters=(1, 1, 1))  # not divisible by 4
    assert e.value.status == 1
    with pytest.raises(CbctError):
        srv.poll(12345)
    srv.close()


def test_poisson_replay_latencies():
    from paper_1001_0599_amd.serving import replay, summarize
    srv = Server(budget_bytes=1e12, max_slots=4, simulated=True)
    arrivals = np.cumsum(np.random.default_rng(51).exponential(0.02, size=20))
    lat, span, _ = replay(srv, arrivals, lambda r: dict(geom=G, iters=(1,), seconds=0.03))
    s = summarize(lat, span)
    assert s["p50_s"] >= 0.03 and s["p99_s"] < 1.0 and s["requests"] == 20
    srv.close()
