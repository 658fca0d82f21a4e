"""Parity of the HIP Siddon projector pair (exact ray-in-voxel lengths) with the FP64 oracle.

Bar: relative L2 <= 2e-5 (float lengths and sums against the FP64 sorted crossings; measured
1e-7 to 7e-6); at full size on sampled rays and voxels that the oracle computes one by one, plus
the adjoint identity."""
import dataclasses

import numpy as np
import pytest
import torch

import cbct_synth as S
import oracle as O
from tests.gpu_util import announce, rel_l2, to_gpu, to_np
from tests.test_gpu_ops import CASES

pytestmark = pytest.mark.gpu
TOL = 2e-5


def _plan(g, levels=1):
    from paper_1001_0599_amd.ops import Plan
    return Plan(g, levels=levels)


@pytest.mark.parametrize("name", list(CASES))
def test_siddon_forward_matches_oracle(name):
    g = CASES[name]
    announce("siddon forward %s %s" % (name, g.vol_shape))
    plan = _plan(g)
    for kind, vol in (("phantom", S.voxelize(g, S.make_phantom(g, 11), 2) if g.nz > 4 else None),
                      ("signed", S.random_volume(g, 5, "normal"))):
        if vol is None:
            continue
        got = to_np(plan.forward_siddon(to_gpu(vol)))
        e = rel_l2(got, O.forward_siddon(g, vol))
        assert e < TOL, (name, kind, e)


@pytest.mark.parametrize("name", list(CASES))
def test_siddon_adjoint_matches_oracle(name):
    g = CASES[name]
    announce("siddon adjoint %s %s" % (name, g.proj_shape))
    plan = _plan(g)
    for kind, y in (("random", S.random_projections(g, 6)), ("signed", S.random_projections(g, 7, "normal"))):
        got = to_np(plan.adjoint_siddon(to_gpu(y)))
        e = rel_l2(got, O.adjoint_siddon(g, y))
        assert e < TOL, (name, kind, e)


def test_siddon_nearly_horizontal_rays():
    """Rays that rise 0.08 mm per 1.5 m (a 2048-row detector over a 352-cell column of 0.25 mm):
    each z crossing lies at z_p lxy / v - t0, a difference of two terms of about 1e3 mm, so the
    crossings are formed in FP64.  Every ray with a tenth of a percent of the largest value or
    more stays within 5e-5 of the FP64 oracle (float crossings left single rays 6e-4 off)."""
    g = dataclasses.replace(CASES["cube32"], nx=8, ny=8, nz=352, hx=2.0, hy=2.0, hz=0.25, nu=16, nv=2048, pu=2.0,
                            pv=0.08, n_views=4, angles=(0.1, 0.9, 2.0, 2.6))
    announce("siddon forward 8x8x352, 4 views x 2048 rows (nearly horizontal rays)")
    plan = _plan(g)
    vol = S.voxelize(g, S.make_phantom(g, 41), 1) + 0.002
    got = to_np(plan.forward_siddon(to_gpu(vol))).astype(np.float64)
    want = O.forward_siddon(g, vol)
    m = np.abs(want) > 1e-3 * np.abs(want).max()
    worst = float((np.abs(got - want)[m] / np.abs(want)[m]).max())
    assert worst < 5e-5, worst
    assert rel_l2(got, want) < 1e-6


@pytest.mark.parametrize("name", ["cube32", "ragged", "anisotropic", "batch128_one"])
def test_siddon_gpu_adjoint_identity(name):
    g = CASES[name]
    plan = _plan(g)
    x = S.random_volume(g, 8, "normal")
    y = S.random_projections(g, 9, "normal")
    a = float(np.vdot(to_np(plan.forward_siddon(to_gpu(x))).astype(np.float64), y))
    b = float(np.vdot(x, to_np(plan.adjoint_siddon(to_gpu(y))).astype(np.float64)))
    assert abs(a - b) / abs(a) < 2e-5, (a, b)


def test_siddon_full_size_sampled():
    """512x512x64, 40 views, 512x384 detector, both multigrid levels: sampled rays and voxels."""
    g = S.config_geometry("wide512x512x64")
    announce("siddon full-size 512x512x64 sampled")
    plan = _plan(g, levels=2)
    rng = np.random.default_rng(2)
    ph = S.make_phantom(g, 21)
    for level in (0, 1):
        gl = S.level_geometry(g, level)
        vol = S.voxelize(gl, ph, 1) + 0.002 * S.random_volume(gl, 3)
        got = to_np(plan.forward_siddon(to_gpu(vol), level=level)).ravel()
        rays = rng.choice(got.size, 3000, replace=False)
        e = rel_l2(got[rays], O.forward_siddon_rays(gl, vol, rays))
        assert e < TOL, ("forward", level, e)
        y = S.random_projections(gl, 11)
        got = to_np(plan.adjoint_siddon(to_gpu(y), level=level)).ravel()
        vox = rng.choice(got.size, 400, replace=False)
        vox = vox[got[vox] != 0][:150]
        e = rel_l2(got[vox], O.adjoint_siddon_voxels(gl, y, vox))
        assert e < TOL, ("adjoint", level, e)


def test_siddon_full_size_adjoint_identity():
    """<P_s x, y> = <x, P_s^T y> at 512x512x64 / 40 views (FP64 inner products of FP32 results)."""
    g = S.config_geometry("wide512x512x64")
    plan = _plan(g)
    for kind, tol in (("uniform", 2e-5), ("normal", 1e-6)):
        x = to_gpu(S.random_volume(g, 12, kind))
        y = to_gpu(S.random_projections(g, 13, kind))
        px = plan.forward_siddon(x).double()
        a = torch.sum(px * y.double()).item()
        b = torch.sum(x.double() * plan.adjoint_siddon(y).double()).item()
        scale = abs(a) if kind == "uniform" else (torch.linalg.norm(px) * torch.linalg.norm(y.double())).item()
        assert abs(a - b) / scale < tol, (kind, a, b)


# a tall thin volume seen by 2048 detector rows: rays enter and leave through the top and bottom
# faces, 352 z cells are too many for the run-summing projector's tables (per-ray walk)
TALL = dataclasses.replace(CASES["cube32"], nx=8, ny=8, nz=352, hx=2.0, hy=2.0, hz=0.25, nu=16, nv=2048, pu=2.0,
                           pv=0.08, n_views=4, angles=(0.1, 0.9, 2.0, 2.6))


def test_siddon_tall_volume():
    g = TALL
    announce("siddon pair on a tall 8x8x352 volume, 2048 rows")
    plan = _plan(g)
    x = S.voxelize(g, S.make_phantom(g, 41), 1) + 0.01 * S.random_volume(g, 43, "normal")
    e = rel_l2(to_np(plan.forward_siddon(to_gpu(x))), O.forward_siddon(g, x))
    assert e < TOL, ("forward", e)
    for seed, kind in ((44, "uniform"), (45, "normal")):
        y = S.random_projections(g, seed, kind)
        e = rel_l2(to_np(plan.adjoint_siddon(to_gpu(y))), O.adjoint_siddon(g, y))
        assert e < TOL, ("adjoint", kind, e)


def test_siddon_deterministic_and_validation():
    from paper_1001_0599_amd import _lib
    g = CASES["ragged"]
    plan = _plan(g)
    x = to_gpu(S.random_volume(g, 14))
    y = to_gpu(S.random_projections(g, 15))
    assert torch.equal(plan.forward_siddon(x), plan.forward_siddon(x))
    assert torch.equal(plan.adjoint_siddon(y), plan.adjoint_siddon(y))
    L = _lib.lib()
    assert L.cbct_forward_siddon(plan.handle, 0, x.data_ptr(), y.data_ptr(), x.data_ptr(), 16, None) == 1
    assert L.cbct_forward_siddon(plan.handle, 1, x.data_ptr(), y.data_ptr(), x.data_ptr(), 4 * x.numel(), None) == 1
    assert L.cbct_adjoint_siddon(plan.handle, 0, y.data_ptr(), None, x.data_ptr(), 1 << 30, None) == 1
    ws = torch.empty(plan.adjoint_siddon_workspace_bytes(0), dtype=torch.uint8, device="cuda")
    assert L.cbct_adjoint_siddon(plan.handle, 0, y.data_ptr(), x.data_ptr(), ws.data_ptr(), 64, None) == 1
