import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


def pytest_collection_modifyitems(config, items):
    # GPU tests are skipped (not failed) on hosts without a GPU
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU on this host")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


def pytest_terminal_summary(terminalreporter):
    # how often the solver parity tests needed the oracle's decisions replayed (FP32 ties)
    mod = sys.modules.get("tests.test_gpu_solver")
    if mod is None or not hasattr(mod, "REPLAYS"):
        return
    try:
        import torch
        if not torch.cuda.is_available():
            return
    except Exception:  # pragma: no cover
        return
    terminalreporter.write_line("solver parity: %d solve(s) replayed an FP32 tie" % len(mod.REPLAYS))
    for shape, iters, q, n, margin in mod.REPLAYS:
        terminalreporter.write_line("  %s iters %s: record %d of %d, oracle margin %.2e" % (shape, iters, q, n, margin))
