"""Edge sizes that select the other kernel paths, against the FP64 oracle on sampled outputs.

* A 2 GiB volume (2048 x 1024 x 256 floats): the run-summing projectors address the volume
  with 32-bit byte offsets, so P and the Siddon P_s take their per-sample / per-ray walks.
* Lines too long for the Siddon profile tables (4096 x 4096 voxels, 2048 detector rows): P_s^T
  takes its per-cell gather.
Bar: relative L2 <= 1e-4 on the sampled rays and voxels."""
import dataclasses

import numpy as np
import pytest
import torch

import cbct_synth as S
import oracle as O
from tests.gpu_util import announce, rel_l2, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-4
G1 = S.config_geometry("cube32")


def _plan(g):
    from paper_1001_0599_amd.ops import Plan
    return Plan(g, levels=1)


def _volume(g, seed):
    rng = np.random.default_rng(seed)
    return rng.random(g.vol_shape, dtype=np.float32)


def test_projectors_2gib_volume():
    g = dataclasses.replace(G1, nx=2048, ny=1024, nz=256, hx=0.25, hy=0.25, hz=0.5, nu=128, nv=64, pu=4.0, pv=1.5,
                            n_views=3, angles=(0.2, 1.4, 2.9))
    assert g.n_vox * 4 >= 2 ** 31
    announce("projectors on a 2048x1024x256 volume (2 GiB)")
    plan = _plan(g)
    x = _volume(g, 3)
    xg = torch.from_numpy(x).cuda()
    rng = np.random.default_rng(4)
    got = to_np(plan.forward(xg)).ravel()
    rays = rng.choice(got.size, 300, replace=False)
    e = rel_l2(got[rays], O.forward_rays(g, x, rays))
    assert e < TOL, ("P", e)
    got = to_np(plan.forward_siddon(xg)).ravel()
    e = rel_l2(got[rays], O.forward_siddon_rays(g, x, rays))
    assert e < TOL, ("P_s", e)


def test_siddon_adjoint_long_lines():
    # a thin slab (one 0.01 mm cell) and 0.01 mm detector rows: a cell meets a few rows
    g = dataclasses.replace(G1, nx=4096, ny=4096, nz=1, hx=0.1, hy=0.1, hz=0.01, nu=16, nv=2048, pu=0.15, pv=0.01,
                            n_views=2, angles=(0.3, 1.9))
    announce("Siddon P^T with 4096 x 4096 voxels and 2048 detector rows")
    plan = _plan(g)
    y = S.random_projections(g, 5)
    got = to_np(plan.adjoint_siddon(torch.from_numpy(y.astype(np.float32)).cuda())).ravel()
    rng = np.random.default_rng(6)
    vox = np.flatnonzero(got)
    vox = rng.choice(vox, min(150, vox.size), replace=False)
    e = rel_l2(got[vox], O.adjoint_siddon_voxels(g, y, vox))
    assert e < TOL, e
