"""bench.py's host-side tools: the counter and kernel-trace summaries (on a small database laid
out as rocprofv3 writes it) and the one-GPU guard."""
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _db(path, counters=(), kernels=()):
    os.makedirs(path, exist_ok=True)
    con = sqlite3.connect(os.path.join(path, "run_results.db"))
    con.execute("create table counters_collection (dispatch_id int, kernel_name text, counter_name text, value real)")
    con.execute("create table kernels (name text, duration int, vgpr_count int, lds_size int, grid_x int, grid_y int, "
                "grid_z int)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", counters)
    con.executemany("insert into kernels values (?, ?, ?, ?, ?, ?, ?)", kernels)
    con.commit()
    con.close()


def _rows(counter, copy, vals):
    """Dispatch records: two small copies and the 256 MiB one, then each kernel's dispatches
    (a counter with two instances, as the per-channel sums arrive)."""
    rows, d = [], 0
    for v in (10.0, copy, 12.0):
        d += 1
        rows += [(d, "__amd_rocclr_copyBuffer(int)", counter, v / 2)] * 2
    for name, per in vals.items():
        for v in per:
            d += 1
            rows += [(d, "void (anonymous namespace)::%s(float const*, int)" % name, counter, v / 2)] * 2
    return rows


def test_counter_summary(tmp_path, capsys):
    kib = 1024.0
    copy_read = 64 * 2 ** 20 * 4  # bytes the calibration copy reads
    names = [pre for _, pre in bench.COUNTER_KERNELS[1:]]
    fetch = {n: [copy_read / kib / 2] for n in names}  # FETCH reads half of what moves (factor 2)
    fetch["k_adj_profiles<true>"] = fetch.pop("k_adj_profiles")
    fetch["k_adj_profiles<true>"] = [1000.0, 3000.0]  # mean 2000 KiB -> 2 x 2000 KiB
    fetch["k_adj_combine"] = [100.0]
    write = {n: [0.0] for n in fetch}
    write["k_adj_combine"] = [50.0]
    write["k_adj_gather_staged<32, 288>"] = write.pop("k_adj_gather_staged")
    write["k_adj_gather_staged<32, 288>"] = [4096.0]
    fetch["k_adj_gather_staged<32, 288>"] = fetch.pop("k_adj_gather_staged")
    hits = {n: [30.0] for n in fetch}
    miss = {n: [10.0] for n in fetch}
    miss["k_adj_profiles<true>"] = [90.0]  # profiles 30 / 120, gather and sum 30 / 40 each
    _db(str(tmp_path / "f"), _rows("FETCH_SIZE", copy_read / kib / 2, fetch))
    _db(str(tmp_path / "w"), _rows("WRITE_SIZE", copy_read / kib, write))
    _db(str(tmp_path / "h"), _rows("TCC_HIT_sum", 1.0, hits) + _rows("TCC_MISS_sum", 1.0, miss))
    bench.counter_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "h"))
    text = capsys.readouterr().out
    assert "copy calibration: FETCH x 2.000, WRITE x 1.000" in text
    kv = dict(line.split(":", 1) for line in text.splitlines() if ":" in line and not line.startswith(" "))
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    # P^T = profiles (2 x 2000 KiB fetched) + gather (2 x copy_read/2 fetched + 4096 KiB written)
    # + view-group sum (2 x 100 KiB fetched + 50 KiB written)
    want = 2 * 2000 * kib + copy_read + 4096 * kib + 2 * 100 * kib + 50 * kib
    assert float(kv["hbm_bytes_per_launch"]) == pytest.approx(want, rel=1e-9)
    assert float(kv["l2_hit_rate"]) == pytest.approx(90.0 / 200.0)
    assert kv["kernel"] == "k_adj_profiles + k_adj_gather_staged + k_adj_combine"
    assert float(kv["forward_hbm_bytes_per_launch"]) == pytest.approx(copy_read, rel=1e-9)
    assert kv["sources_sha256"] == bench.sources_digest(bench.TRAFFIC_SOURCES)


def test_trace_summary(tmp_path, capsys):
    _db(str(tmp_path / "t"), kernels=[
        ("void (anonymous namespace)::k_tv_grad(float const*, float*)", 3000, 24, 32, 2048, 1024, 1),
        ("void (anonymous namespace)::k_tv_grad(float const*, float*)", 1000, 24, 32, 2048, 1024, 1),
        ("void (anonymous namespace)::k_forward_runs<64, 1>(float const*, ColParams const*)", 6000, 48, 37936, 98304,
         40, 1),
    ])
    bench.trace_summary(str(tmp_path / "t"))
    lines = capsys.readouterr().out.splitlines()
    assert lines[1].split()[:2] == ["k_forward_runs<64,", "1>"]
    tv = lines[2].split()
    assert tv[0] == "k_tv_grad" and tv[1] == "[2048x1024x1]"
    assert tv[2:7] == ["2", "0.004", "2.00", "1.00", "3.00"]
    assert lines[-1] == "all kernels: 0.010 ms"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_sq_summary(tmp_path, capsys):
    """VALU-at-peak = SQ_INSTS_VALU / (256 CUs x 2.4 GHz); its share of the kernel's duration."""
    rows = []
    n_valu = 256 * 2.4e9 * 500e-6  # 500 us of VALU issue at peak
    for d, (cn, v) in enumerate([("SQ_INSTS_VALU", n_valu), ("SQ_INSTS_LDS", 1000.0), ("SQ_LDS_BANK_CONFLICT", 500.0),
                                 ("SQ_ACTIVE_INST_VALU", 1.0), ("SQ_ACTIVE_INST_LDS", 1.0), ("SQ_BUSY_CYCLES", 1.0),
                                 ("SQ_WAVE_CYCLES", 1.0), ("SQ_WAVES", 1.0)]):
        rows += [(1, "void (anonymous namespace)::k_adj_gather_staged<32, 320>(float const*)", cn, v / 2)] * 2
    _db(str(tmp_path / "s"), rows, kernels=[
        ("void (anonymous namespace)::k_adj_gather_staged<32, 320>(float const*)", 1_000_000, 72, 52120, 1, 1, 1)])
    bench.sq_summary(str(tmp_path / "s"))
    line = [ln for ln in capsys.readouterr().out.splitlines() if ln.strip().startswith("k_adj_gather_staged")][0]
    f = line.split()
    assert float(f[1]) == pytest.approx(n_valu, rel=1e-3)
    assert float(f[4]) == pytest.approx(0.5)            # bank-conflict cycles per LDS instruction
    assert float(f[5]) == pytest.approx(1000.0)         # duration, us
    assert float(f[6]) == pytest.approx(500.0, rel=1e-3)  # VALU at peak, us
    assert f[7] == "50%"
