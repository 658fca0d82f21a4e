"""cbct_tv_energy_grad_noalloc (no device allocation, partial sums in the library's per-device
scratch array) against cbct_tv_energy_grad (caller workspace) through the C ABI: the same TV sum
and gradient, bitwise (the same kernels and partial-sum layout), on two calls in a row, the
second on a smaller volume (the scratch keeps the first call's contents)."""
import ctypes as C
import dataclasses

import numpy as np
import pytest
import torch

import cbct_synth as S
from tests.gpu_util import announce, to_gpu

pytestmark = pytest.mark.gpu


def _workspace_version(L, plan, level, f, eps):
    n = C.c_size_t()
    assert L.cbct_tv_energy_grad_workspace_size(plan.handle, C.byref(n)) == 0
    ws = torch.empty(int(n.value), dtype=torch.uint8, device=f.device)
    g = torch.empty_like(f)
    h = C.c_double()
    st = L.cbct_tv_energy_grad(plan.handle, level, eps, f.data_ptr(), g.data_ptr(), C.byref(h), ws.data_ptr(),
                               int(n.value), torch.cuda.current_stream().cuda_stream)
    assert st == 0, L.cbct_last_error()
    return h.value, g


def _noalloc_version(L, plan, level, f, eps):
    g = torch.empty_like(f)
    h = C.c_double()
    st = L.cbct_tv_energy_grad_noalloc(plan.handle, level, eps, f.data_ptr(), g.data_ptr(), C.byref(h),
                                       torch.cuda.current_stream().cuda_stream)
    assert st == 0, L.cbct_last_error()
    return h.value, g


def test_noalloc_tv_energy_grad_equals_workspace_version():
    from paper_1001_0599_amd import _lib
    from paper_1001_0599_amd.ops import Plan
    L = _lib.lib()
    base = S.config_geometry("cube32")
    g = dataclasses.replace(base, nx=96, ny=80, nz=48, hx=1.0, hy=1.5, hz=2.5)
    plan = Plan(g, levels=2)
    eps = 1e-5
    # first call: the fine level; second call: the coarse level (a smaller grid, fewer partials)
    for level, seed in ((0, 3), (1, 4)):
        shape = plan.vol_shape(level)
        announce("no-alloc TV energy/grad, level %d %s" % (level, shape))
        f = to_gpu(0.02 * np.random.default_rng(seed).uniform(size=shape))
        want_sum, want_grad = _workspace_version(L, plan, level, f, eps)
        got_sum, got_grad = _noalloc_version(L, plan, level, f, eps)
        torch.cuda.synchronize()
        assert got_sum == want_sum, (level, got_sum, want_sum)
        assert torch.equal(got_grad, want_grad), level
    # the energy alone (no gradient) as well
    f = to_gpu(0.02 * np.random.default_rng(5).uniform(size=plan.vol_shape(1)))
    h = C.c_double()
    assert L.cbct_tv_energy_grad_noalloc(plan.handle, 1, eps, f.data_ptr(), None, C.byref(h),
                                         torch.cuda.current_stream().cuda_stream) == 0
    assert h.value == _workspace_version(L, plan, 1, f, eps)[0]


def test_noalloc_rejects_bad_arguments():
    from paper_1001_0599_amd import _lib
    from paper_1001_0599_amd.ops import Plan
    L = _lib.lib()
    plan = Plan(S.config_geometry("cube32"))
    f = torch.zeros(plan.vol_shape(0), device="cuda")
    h = C.c_double()
    s = torch.cuda.current_stream().cuda_stream
    assert L.cbct_tv_energy_grad_noalloc(plan.handle, 1, 1e-5, f.data_ptr(), None, C.byref(h), s) == 1  # bad level
    assert L.cbct_tv_energy_grad_noalloc(plan.handle, 0, 0.0, f.data_ptr(), None, C.byref(h), s) == 1  # eps <= 0
    assert L.cbct_tv_energy_grad_noalloc(None, 0, 1e-5, f.data_ptr(), None, C.byref(h), s) == 1
