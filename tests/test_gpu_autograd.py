"""P and P^T as autograd Functions (the differentiable-projector workload).

Batch of 8 seeded 128^3 phantoms (2 mm), 60 views, 256x192 detector (2 mm), SAD 1000 /
SDD 1500; loss L(f) = sum_b ||P f_b - y_b||^2 + lambda sum_b S(f_b), S = sum sqrt(|D f|^2 + eps^2),
evaluated at f_b = clip(f0_b + N(0, 0.002^2), 0).  Checks: the autograd gradient against the FP64
oracle's 2 P^T (P f - y) + lambda dS/df (one volume of the batch, rel-L2 1e-4); directional
central differences (h = 1e-3, loss accumulated in FP64) along 4 seeded smooth directions of unit
infinity-norm; the Functions' backward is the hand-written adjoint."""
import numpy as np
import pytest
import torch

import cbct_synth as S
import oracle as O
from tests.gpu_util import announce, rel_l2, to_gpu, to_np

pytestmark = pytest.mark.gpu

CFG = S.CONFIGS["batch8x128"]
G = CFG["geometry"]
LAM = CFG["lam"]
EPS = 1e-5


@pytest.fixture(scope="module")
def batch():
    from paper_1001_0599_amd.ops import Plan
    announce("autograd batch: 8 x 128^3, 60 views")
    plan = Plan(G)
    rng = np.random.default_rng(CFG["perturb_seed"])
    fs, ys = [], []
    for b, seed in enumerate(CFG["phantom_seeds"]):
        ph = S.make_phantom(G, seed)
        f0 = S.voxelize(G, ph, 1)
        fs.append(np.clip(f0 + rng.normal(0.0, 0.002, f0.shape), 0.0, None))
        ys.append(S.poisson_log(S.analytic_projections(G, ph), CFG["I0"], CFG["noise_seed"] * 100 + b))
    return plan, np.stack(fs), np.stack(ys)


def _loss(plan, f, y):
    from paper_1001_0599_amd.autograd import project, tv_sum
    r = project(f, plan).double() - y.double()
    return (r * r).sum() + LAM * tv_sum(f, plan, EPS)


def test_gradient_matches_oracle(batch):
    plan, fs, ys = batch
    f = to_gpu(fs).requires_grad_(True)
    y = to_gpu(ys)
    _loss(plan, f, y).backward()
    g0 = to_np(f.grad[0])
    # oracle gradient of volume 0 (FP64): 2 P^T (P f - y) + lambda N dR/df
    f0 = to_np(f.detach()[0])
    y0 = to_np(y[0])
    want = 2.0 * O.adjoint(G, O.forward(G, f0) - y0) + LAM * G.n_vox * O.tv_grad(G, f0, EPS)
    assert rel_l2(g0, want) < 1e-4


def _smooth_direction(rng, shape):
    """unit-infinity-norm direction made of a few random Gaussian blobs (keeps TV differentiable at h)"""
    z, y, x = np.meshgrid(*[np.linspace(-1, 1, n) for n in shape], indexing="ij")
    v = np.zeros(shape)
    for _ in range(5):
        c = rng.uniform(-0.7, 0.7, 3)
        s = rng.uniform(0.15, 0.4)
        v += rng.choice([-1.0, 1.0]) * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * s * s))
    return v / np.abs(v).max()


def test_directional_finite_differences(batch):
    plan, fs, ys = batch
    f = to_gpu(fs).requires_grad_(True)
    y = to_gpu(ys)
    _loss(plan, f, y).backward()
    grad = f.grad.double()
    rng = np.random.default_rng(CFG["direction_seed"])
    h = 1e-3
    for q in range(4):
        v = to_gpu(np.stack([_smooth_direction(rng, G.vol_shape) for _ in range(fs.shape[0])]))
        with torch.no_grad():
            lp = _loss(plan, f.detach() + h * v, y).item()
            lm = _loss(plan, f.detach() - h * v, y).item()
        fd = (lp - lm) / (2 * h)
        an = float((grad * v.double()).sum())
        assert abs(fd - an) / abs(an) < 2e-3, (q, fd, an)


def test_backward_is_the_adjoint(batch):
    """<P f, w> = <f, P^T w> through the Functions, and grad of <P f, w> equals P^T w."""
    from paper_1001_0599_amd.autograd import backproject, project
    plan, fs, ys = batch
    f = to_gpu(fs[:2]).requires_grad_(True)
    w = to_gpu(np.random.default_rng(3).standard_normal(ys[:2].shape))
    (project(f, plan) * w).sum().backward()
    pt = backproject(w, plan)
    assert torch.equal(f.grad, pt)
    yv = w.clone().requires_grad_(True)
    (backproject(yv, plan) * f.detach()).sum().backward()
    assert torch.equal(yv.grad, project(f.detach(), plan))
